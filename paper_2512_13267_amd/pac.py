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

The gate has two parts.  The spread gate flags a particle when the
ensemble's spread exceeds threshold x max(|mean|, floor); its floor is
calibrated on held-out data of the training distribution (``--calibrate``):
threshold x floor is the spread that 99% of in-distribution rows stay below
(0.0176 in surrogate output units on 44,960 rows, so floor = 0.35), and the
gate reacts to disagreement beyond the ordinary rather than to rows whose
predicted stress is near zero (the relative test alone flags 0.8% of
in-distribution rows, but every particle of a flow at rest).  The members
were trained on the same data and extrapolate alike, so their spread stays
small where the inputs leave the training range; the input-range gate
flags a particle whose current gradient has a Frobenius norm above the
0.9999 quantile of the training set's (train.input_quantile: 0.353 for the
packaged weights).  In this flow the surrogate's error beyond the DPD
noise sits mostly in the particles next to the cylinder, whose shear rates
reach twice that bound.

Command line: ``python -m paper_2512_13267_amd.pac [--steps 500]
[--avg 100,400] [--runs dpd,dpd2,surrogate] [--out FILE]``;
``--calibrate`` prints the in-distribution floor.
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
GATE_FLOOR = 0.35  # surrogate output units: the in-distribution 0.99 quantile of the spread / GATE_THRESHOLD
GATE_INPUT_Q = 0.9999  # input-range gate: this quantile of the training set's gradient norms
GATE_WARM = 0.9  # warm band: boxes of particles above this fraction of the bound stay live, unused
HOLD = 10
# history samples a restored micro-domain relives (on entry to DPD and after a
# thin cell): at 31 the boxes next to the cylinder, under shear rates up to
# 0.7, thin again during their own replays (1958 restores in the surrogate
# run against 193 at 10), with the same stress error
REPLAY = 10


def gate_max_grad(q=GATE_INPUT_Q):
    """The input-range bound of the packaged weights' training set."""
    from . import train

    return train.input_quantile(q, **surrogate.TRAINED_DATA)


def build(mode, seed_k=41, n_lattice=64, n_particles=4000, equil=500, k_micro=50, threshold=GATE_THRESHOLD,
          floor=GATE_FLOOR, hold=HOLD, replay=REPLAY, weights=None, max_grad=None, warm_frac=GATE_WARM):
    """max_grad: the input-range gate's bound (None: gate_max_grad() for the
    packaged weights, 0 for other weights; 0 disables it)."""
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
    if max_grad is None:
        max_grad = gate_max_grad() if weights is None else 0.0
    hy = lhmm.Hybrid(s, m, sur, phi=np.full(nm, phi_feature(PHI), dtype=np.float32),
                     mode="surrogate" if mode == "surrogate" else "dpd", k_micro=k_micro, hold=hold, replay=replay,
                     threshold=threshold, floor=floor, grad_scale=gscale, stress_scale=sscale, max_grad=max_grad,
                     warm_frac=warm_frac if max_grad > 0 else 0.0)
    torch.cuda.synchronize()
    return {"mac": mac, "micro": m, "sph": s, "sur": sur, "hy": hy, "nm": nm, "max_grad": max_grad}


def close(ctx):
    ctx["hy"].close()
    for k in ("sur", "micro", "sph"):
        if ctx[k] is not None:
            ctx[k].close()


def run(ctx, steps, avg, log=print, label=""):
    """Advance `steps` macro steps; returns timing, counters and the mean
    stress over the last `avg` steps (avg: an int, or a list of ints: then a
    dict of means by window)."""
    import torch

    hy = ctx["hy"]
    nm = ctx["nm"]
    windows = sorted({int(a) for a in (avg if isinstance(avg, (list, tuple)) else [avg])})
    longest = windows[-1]
    partial = {}  # mean over [steps - longest, steps - a) for the shorter windows a
    n_dpd = 0
    entered = 0
    resets = 0
    dpd_steps = []  # macro steps (1-based) with any particle on DPD
    n_range = 0
    n_warm = 0
    t0 = time.time()
    st = None
    for k in range(steps):
        if k == steps - longest:
            hy.mean_stress(reset=True)
        for a in windows[:-1]:
            if k == steps - a:
                partial[a] = hy.mean_stress()
        st = hy.step()
        n_dpd += st["n_dpd"]
        if st["n_dpd"]:
            dpd_steps.append(k + 1)
        n_range += st["n_out_of_range"]
        n_warm += st["n_warm"]
        entered += st["n_entered"]
        resets += st["n_reset"]
        if (k + 1) % 50 == 0:
            torch.cuda.synchronize()
            log(f"  {label} macro step {k + 1}/{steps}: {time.time() - t0:.1f} s, on DPD {st['n_dpd']}/{nm}, "
                f"resets so far {resets}", flush=True)
    torch.cuda.synchronize()
    secs = time.time() - t0
    full = hy.mean_stress()
    means = {longest: full}
    for a in windows[:-1]:
        # the last a steps: the long window's sum less its first longest - a steps
        means[a] = (longest * full - (longest - a) * partial[a]) / a
    out = {"steps": steps, "seconds": secs, "macro_steps_per_s": steps / secs,
           "micro_box_steps": st["micro_box_steps"], "fallback_rate": n_dpd / (steps * nm),
           "entered": entered, "resets": resets, "out_of_range_rate": n_range / (steps * nm),
           "warm_rate": n_warm / (steps * nm),
           "macro_steps_with_dpd": len(dpd_steps),
           "last_macro_step_with_dpd": dpd_steps[-1] if dpd_steps else 0}
    return out, (means if isinstance(avg, (list, tuple)) else full)


def calibrate_floor(threshold=GATE_THRESHOLD, n_boxes=512, n_macro=120, max_rate=0.01, seed_k=99, weights=None,
                    log=print):
    """The smallest gate floor for which at most `max_rate` of held-out rows
    of the training distribution (fresh micro-DPD data, seeds never used in
    training) are flagged.  Returns the floor and the spread statistics."""
    import torch

    from . import train

    X, T, _, _, info = train.generate(n_boxes, n_macro, equil=300, seed_k=seed_k, log=log)
    members, nh, _, _ = surrogate.load_trained(weights or surrogate.TRAINED)
    sur = surrogate.Surrogate(members, X.shape[1], nh, 3, max_batch=4096)
    spread, norm = [], []
    for k in range(0, X.shape[0], 4096):
        Y = sur.forward(X[k:k + 4096].contiguous())
        mu = Y.mean(dim=0)
        spread.append(((Y - mu) ** 2).mean(dim=0).mean(dim=1).sqrt())
        norm.append(mu.norm(dim=1))
    sur.close()
    spread = torch.cat(spread).double().cpu().numpy()
    norm = torch.cat(norm).double().cpu().numpy()
    # flagged at floor f where spread > threshold max(norm, f): rows with
    # spread <= threshold norm never are; the others are for f < spread / threshold
    # the floor: spread / threshold at the in-distribution quantile 1 - max_rate,
    # so a flagged row's spread exceeds both threshold x |mean| and what
    # (1 - max_rate) of the training distribution's rows show
    floor = float(np.quantile(spread, 1.0 - max_rate)) / threshold
    rate_at = lambda f: float(np.mean(spread > threshold * np.maximum(norm, f)))
    return {"floor": floor, "threshold": threshold, "max_rate": max_rate, "rows": int(spread.size),
            "flag_rate_at_floor": rate_at(floor), "flag_rate_without_floor": rate_at(0.0),
            "spread_quantiles": {q: float(np.quantile(spread, q)) for q in (0.5, 0.9, 0.99, 0.999)},
            "mean_norm_median": float(np.median(norm)), "samples": info["samples"]}


def deviatoric(sigma):
    tr3 = sigma[:, :3].sum(axis=1) / 3.0
    return np.stack([sigma[:, 0] - tr3, sigma[:, 3], sigma[:, 1] - tr3], axis=1)


def compare(a, b, nm):
    da, db = deviatoric(a[:nm]), deviatoric(b[:nm])
    return float(np.linalg.norm(da - db) / np.linalg.norm(db))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--avg", default="100", help="comma-separated averaging windows (macro steps)")
    ap.add_argument("--runs", default="dpd,dpd2,surrogate")
    ap.add_argument("--out", default=None)
    ap.add_argument("--weights", default=None, help="surrogate weights (default: the packaged ones)")
    ap.add_argument("--thresholds", default=str(GATE_THRESHOLD),
                    help="comma-separated gate thresholds, one surrogate run each")
    ap.add_argument("--floor", type=float, default=GATE_FLOOR)
    ap.add_argument("--hold", type=int, default=HOLD)
    ap.add_argument("--calibrate", action="store_true", help="print the in-distribution gate floor and exit")
    ap.add_argument("--replay", type=int, default=REPLAY)
    ap.add_argument("--warm", type=float, default=GATE_WARM, help="warm band as a fraction of max_grad (0: none)")
    ap.add_argument("--max-grad", type=float, default=None,
                    help="input-range gate bound (default: the packaged weights' training quantile; 0 disables)")
    ap.add_argument("--means-out", default=None, help="save the runs' mean stresses (npz)")
    ap.add_argument("--ref", default=None, help="npz of earlier dpd / dpd2 means to compare against")
    args = ap.parse_args(argv)
    import torch

    if not torch.cuda.is_available():
        raise SystemExit("needs the GPU")
    if args.calibrate:
        cal = calibrate_floor(threshold=float(args.thresholds.split(",")[0]), weights=args.weights)
        print(json.dumps(cal), flush=True)
        if args.out:
            with open(args.out, "w") as f:
                json.dump(cal, f, indent=1)
        return
    windows = [int(a) for a in args.avg.split(",")]
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
                    replay=args.replay, weights=args.weights, max_grad=args.max_grad, warm_frac=args.warm)
        print(f"{name}: {ctx['nm']} micro-domains", flush=True)
        res[name], means[name] = run(ctx, args.steps, windows, label=name)
        res[name]["n_mobile"] = ctx["nm"]
        if mode == "surrogate":
            res[name]["gate"] = {"threshold": th, "floor": args.floor, "max_grad": ctx["max_grad"], "warm": args.warm,
                                 "hold": args.hold, "replay": args.replay}
        print(json.dumps({name: res[name]}), flush=True)
        close(ctx)
    nm = next(iter(res.values()))["n_mobile"]
    if args.means_out:
        np.savez(args.means_out, **{f"{name}_{w}": means[name][w] for name in means for w in windows})
    if args.ref:
        ref = np.load(args.ref)
        for name in ("dpd", "dpd2"):
            if name not in means and all(f"{name}_{w}" in ref for w in windows):
                means[name] = {w: ref[f"{name}_{w}"] for w in windows}
                res.setdefault(name, {"n_mobile": nm, "from": args.ref})
    if "dpd" in means:
        for name in means:
            if name != "dpd":
                res[name]["stress_rel_l2_vs_dpd"] = {w: compare(means[name][w], means["dpd"][w], nm) for w in windows}
        for name in names:
            if name.startswith("surrogate") and "macro_steps_per_s" in res["dpd"]:
                res[name]["speedup_vs_dpd"] = res[name]["macro_steps_per_s"] / res["dpd"]["macro_steps_per_s"]
        if "dpd2" in means:
            # against the mean of the two DPD runs: half the noise variance of one
            for name in names:
                if name.startswith("surrogate"):
                    res[name]["stress_rel_l2_vs_dpd_mean"] = {
                        w: compare(means[name][w], 0.5 * (means["dpd"][w] + means["dpd2"][w]), nm) for w in windows}
    print(json.dumps(res), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
