"""Surrogate-in-the-loop LHMM on the flow past a periodic array of
cylinders, against all-DPD LHMM on the same problem.

Problem: ``inputs.cylinder_array`` (64 x 64 SPH lattice in the unit cell,
cylinder of radius 0.2, uniform body force; ~3.6k mobile particles), each
mobile particle owning a 4000-particle micro-domain of polymer fraction 0.1
(equilibrated at rest).  Runs:

* ``dpd``: every micro-domain advances 50 micro steps per macro step;
* ``dpd2``: the same with another random-force seed (the DPD noise floor);
* ``surrogate``: the trained ensemble supplies the stress, the gate sends
  particles whose members disagree to DPD (restored and replayed).

Reported per run: macro steps/s (wall clock around the steps, device
synchronised), micro box-steps, fallback rate; and the relative L2 error of
the per-particle in-plane deviatoric stress averaged over the last
``avg`` macro steps, surrogate versus ``dpd`` (and versus the mean of
``dpd`` and ``dpd2``), next to ``dpd2`` versus ``dpd``.

Command line: ``python -m paper_2512_13267_amd.pac [--steps 500] [--avg 100]
[--runs dpd,dpd2,surrogate] [--out FILE]``.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import inputs, lhmm, micro, surrogate
from .train import phi_feature

PHI = 0.1
GATE_THRESHOLD = 0.05
GATE_FLOOR = 1.0  # surrogate output units (targets / stress_scale): ~ the RMS training target
HOLD = 10
REPLAY = 31


def build(mode, seed_k=41, n_lattice=64, n_particles=4000, equil=500, k_micro=50, threshold=GATE_THRESHOLD,
          floor=GATE_FLOOR, hold=HOLD, replay=REPLAY, weights=None):
    import torch

    mac = inputs.cylinder_array(n=n_lattice)
    q = mac.params
    nm = mac.r.shape[0] - q["n_fixed"]
    wl = inputs.lhmm_boxes(nm, n_particles=n_particles, polymer_fraction=PHI, seed_k=seed_k)
    m = micro.from_workload(wl, precision="fp32")
    m.step(torch.zeros((nm, 9), dtype=torch.float64, device="cuda"), equil)
    s = lhmm.Sph(q, mac.r, mac.v)
    members, nh, gscale, sscale = surrogate.load_trained(weights or surrogate.TRAINED)
    sur = None
    if mode == "surrogate":
        sur = surrogate.Surrogate(members, members[0]["W1"].shape[0], nh, 3, max_batch=nm)
    hy = lhmm.Hybrid(s, m, sur, phi=np.full(nm, phi_feature(PHI), dtype=np.float32),
                     mode="surrogate" if mode == "surrogate" else "dpd", k_micro=k_micro, hold=hold, replay=replay,
                     threshold=threshold, floor=floor, grad_scale=gscale, stress_scale=sscale)
    torch.cuda.synchronize()
    return {"mac": mac, "micro": m, "sph": s, "sur": sur, "hy": hy, "nm": nm}


def close(ctx):
    ctx["hy"].close()
    for k in ("sur", "micro", "sph"):
        if ctx[k] is not None:
            ctx[k].close()


def run(ctx, steps, avg, log=print, label=""):
    """Advance `steps` macro steps; returns timing, counters and the mean
    stress over the last `avg` steps."""
    import torch

    hy = ctx["hy"]
    nm = ctx["nm"]
    n_dpd = 0
    entered = 0
    resets = 0
    t0 = time.time()
    st = None
    for k in range(steps):
        if k == steps - avg:
            hy.mean_stress(reset=True)
        st = hy.step()
        n_dpd += st["n_dpd"]
        entered += st["n_entered"]
        resets += st["n_reset"]
        if (k + 1) % 50 == 0:
            torch.cuda.synchronize()
            log(f"  {label} macro step {k + 1}/{steps}: {time.time() - t0:.1f} s, on DPD {st['n_dpd']}/{nm}, "
                f"resets so far {resets}", flush=True)
    torch.cuda.synchronize()
    secs = time.time() - t0
    mean = hy.mean_stress()
    return {"steps": steps, "seconds": secs, "macro_steps_per_s": steps / secs,
            "micro_box_steps": st["micro_box_steps"], "fallback_rate": n_dpd / (steps * nm),
            "entered": entered, "resets": resets}, mean


def deviatoric(sigma):
    tr3 = sigma[:, :3].sum(axis=1) / 3.0
    return np.stack([sigma[:, 0] - tr3, sigma[:, 3], sigma[:, 1] - tr3], axis=1)


def compare(a, b, nm):
    da, db = deviatoric(a[:nm]), deviatoric(b[:nm])
    return float(np.linalg.norm(da - db) / np.linalg.norm(db))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--avg", type=int, default=100)
    ap.add_argument("--runs", default="dpd,dpd2,surrogate")
    ap.add_argument("--out", default=None)
    ap.add_argument("--weights", default=None, help="surrogate weights (default: the packaged ones)")
    ap.add_argument("--thresholds", default=str(GATE_THRESHOLD),
                    help="comma-separated gate thresholds, one surrogate run each")
    ap.add_argument("--floor", type=float, default=GATE_FLOOR)
    ap.add_argument("--hold", type=int, default=HOLD)
    args = ap.parse_args(argv)
    import torch

    if not torch.cuda.is_available():
        raise SystemExit("needs the GPU")
    res, means = {}, {}
    names = []
    for name in args.runs.split(","):
        if name == "surrogate":
            names += [f"surrogate@{th}" for th in args.thresholds.split(",")]
        else:
            names.append(name)
    for name in names:
        mode = "surrogate" if name.startswith("surrogate") else "dpd"
        th = float(name.split("@")[1]) if "@" in name else GATE_THRESHOLD
        ctx = build(mode, seed_k=42 if name == "dpd2" else 41, threshold=th, floor=args.floor, hold=args.hold,
                    weights=args.weights)
        print(f"{name}: {ctx['nm']} micro-domains", flush=True)
        res[name], means[name] = run(ctx, args.steps, args.avg, label=name)
        res[name]["n_mobile"] = ctx["nm"]
        print(json.dumps({name: res[name]}), flush=True)
        close(ctx)
    nm = next(iter(res.values()))["n_mobile"]
    if "dpd" in means:
        for name in means:
            if name != "dpd":
                res[name]["stress_rel_l2_vs_dpd"] = compare(means[name], means["dpd"], nm)
        for name in names:
            if name.startswith("surrogate"):
                res[name]["speedup_vs_dpd"] = res[name]["macro_steps_per_s"] / res["dpd"]["macro_steps_per_s"]
        if "dpd2" in means:
            # against the mean of the two DPD runs: half the noise variance of one
            ref = 0.5 * (means["dpd"] + means["dpd2"])
            for name in names:
                if name.startswith("surrogate"):
                    res[name]["stress_rel_l2_vs_dpd_mean"] = compare(means[name], ref, nm)
    print(json.dumps(res), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
