"""Virtual rheometer: steady simple-shear sweeps of micro-boxes and their
Carreau-Yasuda description (Section "Rheological characterization";
Appendix "Carreau-Yasuda Model Details", Eq. Yasuda; Appendix "Normal
Stress Coefficients and Relaxation Time Definitions", Eqs. psi1_appendix,
tau0_def, tau0_def_appendix).

One batched engine call shears every box of a sweep at once: each shear
rate gets `replicas` independent boxes (own random start and random-force
stream), all are first driven to steady state, then the mean Irving-Kirkwood
stress of a second call is the measurement.  Per rate:
  eta(g)     = sigma_xy / g                   (shear viscosity)
  N1(g)      = sigma_xx - sigma_yy            (first normal stress difference)
  psi1(g)    = N1 / g^2                        (Eq. psi1_appendix)
  lambda(g)  = 0.5 psi1 / eta                  (Eq. tau0_def)
with standard errors over the replicas, and the Carreau-Yasuda fit
  eta(g) = eta_inf + (eta0 - eta_inf) [1 + (lam g)^a]^((n - 1) / a)
by least squares in log eta.  Stresses are the engine's (tension positive,
total = kinetic + pair + bond parts).

Two micro models: the engine's 3-D boxes (DPD with FENE chains at density
3), and --planar, the paper's 2-D melt (Tab. 1 parameters, n = 4 per unit
area, no solvent) held in the plane z = 0 of a periodic cell and sheared
homogeneously.  With --afbc the planar melt fills the paper's own
micro-domain instead (Tab. 2: 76 x 76, core 24, boundary-condition region
13, buffer 13): the cell stays fixed, the shear is imposed on the
boundary-condition ring (Eq. micro_bc) and the stress is the core's
Irving-Kirkwood stress.  Planar Carreau-Yasuda parameters are compared with
the paper's table (PAPER_CY).

Command line: ``python -m paper_2512_13267_amd.rheometer [--planar | --afbc]
[--rates ...] [--replicas 16] [--chain-len 10] [--edge E] [--equil 5000]
[--steps 20000] [--zeta 10] [--out FILE]``; ``--report a.json,b.json --md FILE`` writes
a summary of earlier runs.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import inputs

# Carreau-Yasuda parameters the paper fits to its 2-D melts
# (Tab. yasuda_params): N_d -> (eta0, eta_inf, lambda, a, n)
PAPER_CY = {4: (13.20, 0.0, 23.50, 0.71, 0.60), 8: (34.29, 3.15, 89.75, 0.95, 0.37),
            16: (173.18, 4.45, 353.48, 0.55, 0.18), 32: (242.83, 4.81, 1307.88, 1.23, 0.29)}


def carreau_yasuda(gdot, eta0, eta_inf, lam, a, n):
    """Eq. Yasuda."""
    g = np.asarray(gdot, dtype=np.float64)
    return eta_inf + (eta0 - eta_inf) * (1.0 + (lam * g) ** a) ** ((n - 1.0) / a)


def fit_carreau_yasuda(gdot, eta, weights=None) -> dict:
    """Least-squares fit of Eq. Yasuda to eta(gdot) in log eta (weights:
    1 / relative standard error, optional), with 0 <= eta_inf < eta0,
    0.05 <= a <= 20 and 0 <= n <= 1.  Returns the five parameters and the
    RMS relative residual."""
    from scipy.optimize import least_squares

    g = np.asarray(gdot, dtype=np.float64)
    e = np.asarray(eta, dtype=np.float64)
    if g.shape != e.shape or g.size < 5 or np.any(g <= 0) or np.any(e <= 0):
        raise ValueError("need at least five positive (rate, viscosity) points")
    w = np.ones_like(e) if weights is None else np.asarray(weights, dtype=np.float64)
    order = np.argsort(g)
    e_top = float(e.max())
    g_mid = float(np.sqrt(g[order[0]] * g[order[-1]]))

    # x = (log eta0, logit(eta_inf / eta0), log lam, log a, n)
    def params(x):
        eta0 = float(np.exp(x[0]))
        return eta0, eta0 / (1.0 + float(np.exp(-x[1]))), float(np.exp(x[2])), float(np.exp(x[3])), float(x[4])

    def resid(x):
        with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
            r = w * (np.log(carreau_yasuda(g, *params(x))) - np.log(e))
        return np.where(np.isfinite(r), r, 1e6)

    lo = [math.log(e_top) - 10.0, -30.0, math.log(1.0 / g_mid) - 25.0, math.log(0.05), 0.0]
    hi = [math.log(e_top) + 10.0, 30.0, math.log(1.0 / g_mid) + 25.0, math.log(20.0), 1.0]
    best = None
    for ratio, lam_shift, a0, n0 in ((0.1, 0.0, 1.0, 0.5), (1e-4, 1.0, 1.0, 0.3), (0.3, -1.0, 2.0, 0.5),
                                      (1e-4, 3.0, 0.7, 0.3), (0.05, -3.0, 1.5, 0.2)):
        start = np.array([math.log(e_top), math.log(ratio / (1.0 - ratio)), math.log(1.0 / g_mid) + lam_shift,
                          math.log(a0), n0])
        r = least_squares(resid, start, bounds=(lo, hi), x_scale="jac", max_nfev=5000)
        if best is None or r.cost < best.cost:
            best = r
    eta0, eta_inf, lam, a, n = params(best.x)
    rel = carreau_yasuda(g, eta0, eta_inf, lam, a, n) / e - 1.0
    # parameters the fit pushed onto a bound are not determined by the data
    names = ("eta0", "eta_inf", "lam", "a", "n")
    at_bounds = [nm for nm, x, l, h in zip(names, best.x, lo, hi) if min(x - l, h - x) < 1e-4 * (h - l)]
    return {"eta0": eta0, "eta_inf": eta_inf, "lam": lam, "a": a, "n": n,
            "rms_rel_residual": float(np.sqrt(np.mean(rel ** 2))), "at_bounds": at_bounds}


def normal_stress_and_relaxation(gdot, sigma):
    """psi1 = N1 / g^2 (Eq. psi1_appendix) and lambda = 0.5 psi1 / eta
    (Eq. tau0_def) from mean stresses (rows (xx, yy, zz, xy, xz, yz))."""
    g = np.asarray(gdot, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    eta = s[:, 3] / g
    n1 = s[:, 0] - s[:, 1]
    psi1 = n1 / g ** 2
    return eta, n1, psi1, 0.5 * psi1 / eta


PLANAR_THICKNESS = inputs.PLANAR_THICKNESS
# the paper's micro-domain (Tab. 2): total 76, core 24, boundary-condition
# region 13 and buffer 13 on each side -> half-widths of the core and of the
# ring's outer edge
AFBC_EDGE, AFBC_CORE_HALF, AFBC_RING_HALF = 76.0, 12.0, 25.0


def sweep_workload(rates, replicas: int = 16, chain_len: int = 10, edge: float = 10.0, density: float = 3.0,
                   polymer_fraction: float = 1.0, seed_k: int = 60, planar: bool = False,
                   **param_over) -> inputs.Workload:
    """Boxes of a shear sweep: for every rate, `replicas` boxes of chains
    (polymer fraction 1: a melt) under simple shear u_x = rate y.  Cubic
    boxes of the given edge and number density per volume, or (planar) 2-D
    systems of edge x edge at the given density per area, held in the
    plane z = 0 of a cell of z edge PLANAR_THICKNESS, with the paper's
    melt parameters (Tab. 1) unless overridden."""
    if planar:
        p = inputs.paper_melt_params(chain_len=chain_len, seed=inputs.SEED_BASE + seed_k, **param_over)
        N = int(round(density * edge ** 2))
        h = np.diag([edge, edge, PLANAR_THICKNESS])
    else:
        p = inputs.default_params(seed=inputs.SEED_BASE + seed_k, chain_len=chain_len, **param_over)
        N = int(round(density * edge ** 3))
        h = inputs.cubic_cell(edge)
    rng = np.random.default_rng(inputs.SEED_BASE + seed_k)
    n_chains = int(polymer_fraction * N) // chain_len  # whole chains; the rest is solvent
    boxes = []
    for rate in rates:
        for _ in range(replicas):
            s, c = inputs.random_box(rng, h, N, n_chains, chain_len, p["kBT"], p["mass"], planar=planar)
            boxes.append(inputs.BoxInit(s=s, c=c, h=h, n_chains=n_chains, L=inputs.shear_gradient(float(rate)),
                                        edge=edge, phi=polymer_fraction))
    return inputs.Workload("shear_sweep_2d" if planar else "shear_sweep", p, boxes, 0)


def run_sweep(rates, replicas: int = 16, chain_len: int = 10, equil: int = 5000, steps: int = 20000,
              edge: float = 10.0, seed_k: int = 60, planar: bool = False, density: float | None = None,
              afbc=None, zeta: float = 10.0, log=print) -> dict:
    """Shear every box of the sweep for `equil` steps, then average the
    stress over `steps` more; per-rate means and standard errors.  Planar
    sweeps report the 2-D stress (force per length: the cell stress times
    its z edge).  afbc = (core half-width, ring half-width): planar boxes
    with boundary regions, the shear imposed on the ring (relaxation rate
    zeta) and the core's stress measured."""
    import torch

    from . import micro

    rates = np.asarray(rates, dtype=np.float64)
    if density is None:
        density = 4.0 if planar else 3.0
    wl = sweep_workload(rates, replicas, chain_len, edge, density=density, seed_k=seed_k, planar=planar)
    m = micro.from_workload(wl, precision="fp32")
    if afbc is not None:
        if not planar:
            raise ValueError("boundary regions are for the planar melt")
        m.set_afbc(np.tile(np.asarray(afbc, dtype=np.float64), (len(wl.boxes), 1)), zeta=zeta)
    G = torch.tensor(np.stack([b.L for b in wl.boxes]), dtype=torch.float64, device="cuda").contiguous()
    t0 = time.time()
    chunk = 1000
    for k in range(0, equil, chunk):
        m.step(G, min(chunk, equil - k))
        torch.cuda.synchronize()
        log(f"  equilibration under shear: {min(k + chunk, equil)}/{equil} steps, {time.time() - t0:.1f} s",
            flush=True)
    # the mean over several calls of equal length is the mean over all steps
    acc = np.zeros((len(wl.boxes), 6))
    n_calls = 0
    for k in range(0, steps, chunk):
        acc += m.step(G, min(chunk, steps - k)).cpu().numpy() * min(chunk, steps - k)
        n_calls += min(chunk, steps - k)
        log(f"  averaging: {n_calls}/{steps} steps, {time.time() - t0:.1f} s", flush=True)
    flags = m.flags()
    m.close()
    per_box = (acc / n_calls).reshape(len(rates), replicas, 6)
    if planar:
        per_box = per_box * PLANAR_THICKNESS
    mean = per_box.mean(axis=1)
    se = per_box.std(axis=1, ddof=1) / math.sqrt(replicas)
    eta, n1, psi1, lam = normal_stress_and_relaxation(rates, mean)
    out = {"rates": rates.tolist(), "replicas": replicas, "chain_len": chain_len, "edge": edge,
           "dims": 2 if planar else 3, "density": density,
           "afbc": None if afbc is None else {"core_half": afbc[0], "ring_half": afbc[1], "zeta": zeta},
           "equil_steps": equil, "avg_steps": steps, "dt": wl.params["dt"],
           "n_particles": wl.n_particles, "seconds": time.time() - t0,
           "flagged_boxes": int(np.count_nonzero(flags)),
           "eta": eta.tolist(), "eta_se": (se[:, 3] / rates).tolist(),
           "N1": n1.tolist(), "N1_se": np.sqrt(se[:, 0] ** 2 + se[:, 1] ** 2).tolist(),
           "psi1": psi1.tolist(), "lambda": lam.tolist(), "sigma_mean": mean.tolist()}
    cy = sweep_fit(out)
    if cy:
        out["carreau_yasuda"] = cy
    return out


def sweep_fit(res: dict):
    """Carreau-Yasuda fit of a sweep's viscosities, weighted by their
    relative standard errors (None with fewer than five positive points)."""
    rates = np.asarray(res["rates"], dtype=np.float64)
    eta = np.asarray(res["eta"], dtype=np.float64)
    ok = eta > 0
    if ok.sum() < 5:
        return None
    w = 1.0 / np.maximum(np.asarray(res["eta_se"])[ok] / eta[ok], 1e-3)
    return fit_carreau_yasuda(rates[ok], eta[ok], weights=w)


def chain_scaling(chain_lens, lams) -> dict:
    """Power law lambda ~ N_d^b by least squares in log-log (the paper's
    Rouse comparison, Fig. 2(e))."""
    x = np.log(np.asarray(chain_lens, dtype=np.float64))
    y = np.log(np.asarray(lams, dtype=np.float64))
    b, c = np.polyfit(x, y, 1)
    return {"b": float(b), "prefactor": float(math.exp(c))}


def report(results, command: str) -> str:
    """Markdown summary of one or more sweeps (one per chain length)."""
    planar = results[0].get("dims", 3) == 2
    af = results[0].get("afbc")
    if planar and af:
        box = ("Micro-domains: the paper's 2-D melt (Tab. 1: DPD a = 25, gamma = 4.5, kBT = 1, FENE H = 50, "
               "R0 = 1.5, dt = 0.005; n = 4 per unit area, polymer fraction 1) in the paper's micro-domain of "
               "Tab. 2, {edge} x {edge} rc (core {core:g}, boundary-condition region {bc:g}, buffer {buf:g}), held "
               "in the plane z = 0 of a fixed periodic cell of z edge {th} rc; the shear is imposed on the "
               "boundary-condition region (Eq. micro_bc; velocities relax toward the imposed field at rate "
               "zeta = {zeta:g} with thermal noise) and the stress is the core's Irving-Kirkwood stress, 2-D "
               "(times the z edge)").format(edge=results[0]["edge"], core=2 * af["core_half"],
                                            bc=af["ring_half"] - af["core_half"],
                                            buf=results[0]["edge"] / 2 - af["ring_half"], th=PLANAR_THICKNESS,
                                            zeta=af["zeta"])
    elif planar:
        box = ("Boxes: the paper's 2-D melt (Tab. 1: DPD a = 25, gamma = 4.5, kBT = 1, FENE H = 50, R0 = 1.5, "
               "dt = 0.005; n = 4 per unit area, polymer fraction 1), {edge} x {edge} rc periodic, held in the "
               "plane z = 0 of a cell of z edge {th} rc and sheared homogeneously (Lees-Edwards); stresses are 2-D "
               "(the cell stress times its z edge)").format(edge=results[0]["edge"], th=PLANAR_THICKNESS)
    else:
        box = ("Boxes: cubic, edge {edge} rc, density 3, polymer fraction 1 (whole chains, the few leftover "
               "particles solvent), DPD a = 25, gamma = 4.5, kBT = 1, FENE H = 30, R0 = 1.5, dt = 0.01").format(
                   edge=results[0]["edge"])
    L = ["# Virtual rheometer: steady simple shear of DPD/FENE melts", "",
         box + "; every rate has {rep} boxes with their own start and random-force stream, all rates of a chain "
         "length in one batched engine call.  Stress: the engine's Irving-Kirkwood mean (tension positive).".format(
             rep=results[0]["replicas"]), "",
         "Command (MI355X, one GPU):", "", "```", command, "```", ""]
    for r in results:
        L += [f"## N_d = {r['chain_len']} ({r['equil_steps']} steps to steady state, then {r['avg_steps']} "
              f"averaged; {r['n_particles']} particles, {r['seconds']:.1f} s; flagged boxes {r['flagged_boxes']})", "",
              "| rate | eta | SE | N1 | SE | psi1 = N1 / rate^2 | lambda = 0.5 psi1 / eta |", "|---|---|---|---|---|---|---|"]
        for row in zip(r["rates"], r["eta"], r["eta_se"], r["N1"], r["N1_se"], r["psi1"], r["lambda"]):
            L.append("| {:.3g} | {:.4g} | {:.2g} | {:.4g} | {:.2g} | {:.4g} | {:.4g} |".format(*row))
        cy = r.get("carreau_yasuda")
        if cy and "at_bounds" not in cy:
            cy = sweep_fit(r) or cy  # results written before the bound check: the same fit again
        if cy:
            L += ["", "Carreau-Yasuda fit (Eq. Yasuda, weighted by the standard errors): eta0 = {eta0:.4g}, "
                  "eta_inf = {eta_inf:.4g}, lambda = {lam:.4g}, a = {a:.3g}, n = {n:.3g}; RMS relative residual "
                  "{rms_rel_residual:.3g}.".format(**cy)
                  + (" At a bound of the fit (not determined by the data): " + ", ".join(cy["at_bounds"]) + "."
                     if cy.get("at_bounds") else "")]
        if planar and r["chain_len"] in PAPER_CY:
            e0, ei, lam, a, n = PAPER_CY[r["chain_len"]]
            pred = carreau_yasuda(np.asarray(r["rates"]), e0, ei, lam, a, n)
            L += ["", f"The paper's fit for N_d = {r['chain_len']} (Tab. yasuda_params): eta0 = {e0}, "
                  f"eta_inf = {ei}, lambda = {lam}, a = {a}, n = {n}; its curve at the rates above: "
                  + ", ".join(f"{x:.4g}" for x in pred) + "."]
        L.append("")
    fits = [(r["chain_len"], r["carreau_yasuda"]["lam"]) for r in results if r.get("carreau_yasuda")]
    if len(fits) >= 2:
        sc = chain_scaling([f[0] for f in fits], [f[1] for f in fits])
        L += ["## Relaxation time against chain length", "",
              "| N_d | lambda (Carreau-Yasuda) |", "|---|---|"] + [f"| {n} | {lam:.4g} |" for n, lam in fits] + [
              "", f"lambda ~ N_d^b with b = {sc['b']:.3f} (least squares in log-log); the Rouse model gives 2.", ""]
    if not planar:
        L += ["The micro model is the engine's 3-D DPD/FENE model, not the paper's 2-D melt, so these parameters "
              "are not comparable with the paper's table.", ""]
    else:
        rows = [r for r in results if r.get("carreau_yasuda") and r["chain_len"] in PAPER_CY]
        if rows:
            L += ["## Against the paper's table (Tab. yasuda_params)", "",
                  "| N_d | eta0 here / paper | eta_inf here / paper | lambda here / paper | eta at the highest rate "
                  "here / paper's curve |", "|---|---|---|---|---|"]
            for r in rows:
                cy, (e0, ei, lam, a, n) = r["carreau_yasuda"], PAPER_CY[r["chain_len"]]
                g = r["rates"][-1]
                L.append(f"| {r['chain_len']} | {cy['eta0']:.4g} / {e0} | {cy['eta_inf']:.4g} / {ei} | "
                         f"{cy['lam']:.4g} / {lam} | {r['eta'][-1]:.4g} / "
                         f"{float(carreau_yasuda(g, e0, ei, lam, a, n)):.4g} (rate {g:g}) |")
            L.append("")
    return "\n".join(L)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--rates", default="0.01,0.02,0.05,0.1,0.2,0.5,1.0,2.0")
    ap.add_argument("--replicas", type=int, default=16)
    ap.add_argument("--chain-len", type=int, default=10)
    ap.add_argument("--planar", action="store_true", help="the paper's 2-D melt (Tab. 1, n = 4)")
    ap.add_argument("--afbc", action="store_true",
                    help="the 2-D melt in the paper's micro-domain with boundary regions (Tab. 2)")
    ap.add_argument("--zeta", type=float, default=10.0, help="relaxation rate of the boundary-condition region")
    ap.add_argument("--edge", type=float, default=None, help="box edge (default 10, planar 32)")
    ap.add_argument("--equil", type=int, default=5000)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--out", default=None)
    ap.add_argument("--report", default=None, help="comma-separated result files: write a summary, no GPU")
    ap.add_argument("--md", default=None, help="summary file for --report")
    ap.add_argument("--command", default="", help="command line quoted in the summary")
    args = ap.parse_args(argv)
    if args.report:
        results = []
        for path in args.report.split(","):
            with open(path) as f:
                results.append(json.load(f))
        text = report(results, args.command)
        if args.md:
            with open(args.md, "w") as f:
                f.write(text)
        print(text)
        return
    import torch

    if not torch.cuda.is_available():
        raise SystemExit("needs the GPU")
    rates = [float(x) for x in args.rates.split(",")]
    planar = args.planar or args.afbc
    edge = args.edge if args.edge is not None else (AFBC_EDGE if args.afbc else (32.0 if planar else 10.0))
    afbc = (AFBC_CORE_HALF * edge / AFBC_EDGE, AFBC_RING_HALF * edge / AFBC_EDGE) if args.afbc else None
    res = run_sweep(rates, args.replicas, args.chain_len, args.equil, args.steps, edge=edge, planar=planar,
                    afbc=afbc, zeta=args.zeta)
    print(json.dumps(res), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
