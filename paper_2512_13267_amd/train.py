"""Training pipeline of the stress surrogate.

Data: a batch of micro-domains (4000 particles, polymer fraction uniform in
[0.1, 0.3]) advanced by the batched micro-DPD engine under random
gradient histories: each box follows piecewise-constant traceless in-plane
gradients, one per macro step, whose three free entries are independent
Ornstein-Uhlenbeck sequences (correlation CORR_STEPS macro steps) with a
per-box standard deviation GRAD_SD x 10^u, u uniform in AMP_RANGE, so that
slow and fast flows are both covered.  A sample is (the box's last LHMM_SUR_HIST
gradients and its polymer fraction) -> (the in-plane deviatoric micro
stress averaged over the macro step's micro steps), the quantity the
macro momentum equation takes from a micro-domain (Eq. pip).  Every step of
the data path runs in the library: micro steps, history ring, features and
targets.  PyTorch only holds the buffers and shuffles the rows.

A periodic cell under a generic time-varying flow is eventually stretched
until its reduced cell becomes too thin for the cutoff.  Boxes that reach
the LHMM_FLAG_THIN width are returned to their equilibrated snapshot; their
samples count again once LHMM_SUR_HIST macro steps have passed since the
restart, so every kept sample's history window was lived by its box.

Training: every member takes the same minibatches (members differ by their
random initialisation), Adam with a cosine-decayed learning rate, mean
squared error on targets divided by STRESS_SCALE.  Each minibatch row is
replaced by a random image under in-plane rotations and reflections
(lhmm_sur_augment): the micro model is isotropic, so the image is a sample
of the same conditional law.  10 % of the boxes are
held out.  A group of boxes can be run as replicas (same start, same
gradients, different random-force streams) to measure the DPD noise of a
target.

Command line: ``python -m paper_2512_13267_amd.train --out DIR`` writes
``surrogate.npz`` (weights and scales) and ``train_metrics.json``.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from . import _lib, inputs, surrogate
from .micro import from_workload

HIST = _lib.SUR_HIST
N_FEATURES = _lib.SUR_FEATURES
GRAD_SD = 0.05
CORR_STEPS = 10.0
AMP_RANGE = (-1.0, 0.2)
GRAD_SCALE = 1.0 / GRAD_SD     # features hold L / GRAD_SD
STRESS_SCALE = 0.1             # the network predicts deviatoric stress / STRESS_SCALE
K_MICRO = 50
PHI_RANGE = (0.1, 0.3)
RESET_FLAGS = _lib.FLAG_THIN | _lib.FLAG_CELL | _lib.FLAG_BOND | _lib.FLAG_NONFINITE
BAD_FLAGS = _lib.FLAG_CELL | _lib.FLAG_BOND | _lib.FLAG_NONFINITE


def phi_feature(phi):
    """Polymer fraction as fed to the network (centred, unit range)."""
    return (np.asarray(phi, dtype=np.float32) - 0.2) * 10.0


def ou_gradients(n_boxes, n_macro, sd=GRAD_SD, corr=CORR_STEPS, seed=0):
    """(n_macro, n_boxes, 9) piecewise-constant gradients [[a, b, 0], [c, -a, 0], 0]
    with (a, b, c) stationary OU sequences; sd and corr (macro steps): a
    number or one per box."""
    rng = np.random.default_rng(seed)
    rho = np.exp(-1.0 / np.broadcast_to(np.asarray(corr, dtype=np.float64), (n_boxes,)))[:, None]
    sd = np.broadcast_to(np.asarray(sd, dtype=np.float64), (n_boxes,))[:, None]
    x = rng.normal(size=(n_boxes, 3)) * sd
    out = np.zeros((n_macro, n_boxes, 9))
    for t in range(n_macro):
        out[t, :, 0], out[t, :, 1], out[t, :, 3], out[t, :, 4] = x[:, 0], x[:, 1], x[:, 2], -x[:, 0]
        x = rho * x + np.sqrt(1.0 - rho * rho) * sd * rng.normal(size=(n_boxes, 3))
    return out


def gradient_histories(n_unique, n_macro, seed_k=3, amp_range=AMP_RANGE, corr_range=(CORR_STEPS, CORR_STEPS),
                       shear=None):
    """The polymer fractions and gradient sequences of generate's boxes
    (its arguments are described there): phis (n_unique,), G
    (n_macro, n_unique, 9), the per-box amplitudes, correlation times and
    shear amplitudes."""
    rng = np.random.default_rng(inputs.SEED_BASE + seed_k)
    phis_u = rng.uniform(*PHI_RANGE, size=n_unique)
    sd_u = GRAD_SD * 10.0 ** rng.uniform(*amp_range, size=n_unique)
    if corr_range[0] == corr_range[1]:
        corr_u = np.full(n_unique, float(corr_range[0]))
    else:
        rng_c = np.random.default_rng(inputs.SEED_BASE + seed_k + 2)
        corr_u = np.exp(rng_c.uniform(math.log(corr_range[0]), math.log(corr_range[1]), size=n_unique))
    G_u = ou_gradients(n_unique, n_macro, sd=sd_u, corr=corr_u, seed=inputs.SEED_BASE + seed_k + 1)
    shear_sd = np.zeros(n_unique)
    if shear is not None:
        frac, lo, hi = shear
        rng_s = np.random.default_rng(inputs.SEED_BASE + seed_k + 3)
        pick = rng_s.uniform(size=n_unique) < frac
        shear_sd = np.where(pick, GRAD_SD * 10.0 ** rng_s.uniform(lo, hi, size=n_unique), 0.0)
        S = ou_gradients(n_unique, n_macro, sd=shear_sd, corr=corr_u, seed=inputs.SEED_BASE + seed_k + 4)
        G_u[:, :, 1] += S[:, :, 1]
    return phis_u, G_u, sd_u, corr_u, shear_sd


def input_quantile(q, n_boxes, n_macro, seed_k=3, amp_range=AMP_RANGE, corr_range=(CORR_STEPS, CORR_STEPS),
                   shear=None):
    """The q-quantile of the Frobenius norm of the newest gradient over the
    rows of a training set made by generate(n_boxes, n_macro, seed_k, ...)
    (every box from the step its history is full; boxes restored after a
    thin cell drop a few rows, which this ignores).  It bounds the inputs the
    ensemble has seen: the hybrid's input-range gate takes it as max_grad."""
    _, G, _, _, _ = gradient_histories(n_boxes, n_macro, seed_k, amp_range, corr_range, shear)
    G = G[HIST - 1:]
    norm = np.sqrt((G * G).sum(axis=2)).ravel()
    return float(np.quantile(norm, q))


def generate(n_boxes, n_macro, k_micro=K_MICRO, equil=500, seed_k=3, replicas=1, amp_range=AMP_RANGE,
             corr_range=(CORR_STEPS, CORR_STEPS), shear=None, log=print):
    """Run the micro engine and return device tensors X (n, 129), T (n, 3),
    box (n,) int32, step (n,) int32 and a summary dict.  With replicas = R,
    boxes come in groups of R sharing start and gradients.  amp_range: the
    range of u in the per-box amplitude GRAD_SD x 10^u; corr_range: the range
    of the per-box correlation time (log-uniform; one value: fixed); shear =
    (frac, lo, hi): a fraction frac of the boxes also get a simple shear
    along x, an OU sequence of amplitude GRAD_SD x 10^u, u uniform in
    [lo, hi], added to the gradient's xy entry (shear-dominated flows at
    higher rates, as near walls, without the chain stretch of sustained
    strong extension)."""
    import torch

    n_unique = n_boxes // replicas
    phis_u, G_u, sd_u, corr_u, shear_sd = gradient_histories(n_unique, n_macro, seed_k, amp_range, corr_range, shear)
    wl_u = inputs.lhmm_boxes(n_unique, polymer_fraction=phis_u, seed_k=seed_k)
    boxes = [b for b in wl_u.boxes for _ in range(replicas)]
    wl = inputs.Workload("surrogate_data", wl_u.params, boxes, 0)
    phis = np.repeat(phis_u, replicas)
    G_host = np.repeat(G_u, replicas, axis=1)
    t0 = time.time()
    m = from_workload(wl, precision="fp32", rng_ids=list(range(n_boxes)))
    st = m.stream
    dev = torch.device("cuda")
    zero = torch.zeros((n_boxes, 9), dtype=torch.float64, device=dev)
    m.step(zero, equil)
    m.snapshot()
    m.flags(clear=True)
    G = torch.from_numpy(G_host).to(dev)
    ring = torch.zeros((n_boxes, HIST, 4), dtype=torch.float32, device=dev)
    phi_d = torch.from_numpy(phi_feature(phis)).to(dev)
    Xt = torch.empty((n_boxes, N_FEATURES), dtype=torch.float32, device=dev)
    Tt = torch.empty((n_boxes, 3), dtype=torch.float32, device=dev)
    sig = torch.empty((n_boxes, 6), dtype=torch.float64, device=dev)
    cap = n_boxes * max(n_macro - HIST + 1, 1)
    X = torch.empty((cap, N_FEATURES), dtype=torch.float32, device=dev)
    T = torch.empty((cap, 3), dtype=torch.float32, device=dev)
    box_id = torch.empty(cap, dtype=torch.int32, device=dev)
    step_id = torch.empty(cap, dtype=torch.int32, device=dev)
    ids_all = torch.arange(n_boxes, dtype=torch.int32, device=dev)
    age = np.zeros(n_boxes, dtype=np.int64)
    n = 0
    resets = 0
    bad = 0
    with torch.cuda.stream(st):
        for t in range(n_macro):
            g = G[t].contiguous()
            surrogate.push_history(ring, g, t, st, scale=GRAD_SCALE)
            m.step(g, k_micro, out=sig)
            surrogate.features(ring, t, phi_d, Xt, st)
            surrogate.targets(sig, 1.0 / STRESS_SCALE, Tt, st)
            fl = m.flags(clear=True)
            age += 1
            keep = (age >= HIST) & ((fl & BAD_FLAGS) == 0)
            bad += int(((fl & BAD_FLAGS) != 0).sum())
            if keep.any():
                idx = torch.from_numpy(np.nonzero(keep)[0]).to(dev)
                k = idx.numel()
                X[n:n + k] = Xt[idx]
                T[n:n + k] = Tt[idx]
                box_id[n:n + k] = ids_all[idx]
                step_id[n:n + k] = t
                n += k
            reset = np.nonzero(fl & RESET_FLAGS)[0]
            if reset.size:
                m.restore(reset.astype(np.int32))
                age[reset] = 0
                resets += int(reset.size)
            if (t + 1) % 50 == 0:
                torch.cuda.synchronize()
                log(f"  macro step {t + 1}/{n_macro}: {n} samples, {resets} resets, "
                    f"{time.time() - t0:.1f} s", flush=True)
    torch.cuda.synchronize()
    info = {"n_boxes": n_boxes, "replicas": replicas, "n_macro": n_macro, "k_micro": k_micro, "equil": equil,
            "samples": n, "resets": resets, "bad_samples": bad, "seconds": time.time() - t0,
            "grad_sd_range": [float(sd_u.min()), float(sd_u.max())],
            "corr_steps_range": [float(corr_u.min()), float(corr_u.max())],
            "shear": None if shear is None else {"frac": float(shear[0]), "u_range": [float(shear[1]), float(shear[2])],
                                                 "boxes": int(np.count_nonzero(shear_sd))}}
    m.close()
    return X[:n], T[:n], box_id[:n], step_id[:n], info


def evaluate(sur, X, T, batch):
    """Ensemble mean predictions and relative errors on (X, T)."""
    import torch

    means = []
    spreads = []
    for k in range(0, X.shape[0], batch):
        Y = sur.forward(X[k:k + batch].contiguous())
        means.append(Y.mean(dim=0))
        spreads.append(Y.std(dim=0, unbiased=False).pow(2).mean(dim=1).sqrt())
    M = torch.cat(means)
    err = (M - T).double()
    rel = float(err.norm() / T.double().norm())
    comp = [float(err[:, j].norm() / T[:, j].double().norm()) for j in range(3)]
    return M, {"rel_l2": rel, "rel_l2_xx_xy_yy": comp, "rmse_scaled": float(err.pow(2).mean().sqrt()),
               "mean_spread_scaled": float(torch.cat(spreads).mean())}


def train(X, T, box_id, n_members=5, hidden=256, epochs=30, batch=4096, lr=1e-3, seed=0, held_mod=10,
          augment=True, log=print):
    import torch

    dev = X.device
    held = (box_id % held_mod) == 0
    tr = torch.nonzero(~held).flatten()
    te = torch.nonzero(held).flatten()
    members = surrogate.init_members(n_members, N_FEATURES, hidden, 3, seed=inputs.SEED_BASE + 100 + seed)
    sur = surrogate.Surrogate(members, N_FEATURES, hidden, 3, max_batch=batch)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(inputs.SEED_BASE + 200 + seed)
    steps_per_epoch = max(tr.numel() // batch, 1)
    total = steps_per_epoch * epochs
    loss = torch.zeros(n_members, dtype=torch.float32, device=dev)
    acc = torch.zeros(n_members, dtype=torch.float64, device=dev)
    t0 = time.time()
    history = []
    k = 0
    with torch.cuda.stream(sur.stream):
        for ep in range(epochs):
            perm = tr[torch.randperm(tr.numel(), generator=gen).to(dev)]
            acc.zero_()
            for j in range(steps_per_epoch):
                idx = perm[j * batch:(j + 1) * batch]
                rate = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * k / total)))
                Xb, Tb = X[idx].contiguous(), T[idx].contiguous()
                if augment:
                    theta = (torch.rand(idx.numel(), generator=gen) * (2.0 * math.pi)).to(dev)
                    mirror = torch.randint(0, 2, (idx.numel(),), generator=gen, dtype=torch.int32).to(dev)
                    surrogate.augment(Xb, Tb, theta, mirror, sur.stream)
                sur.train_step(Xb, Tb, rate, loss)
                acc += loss
                k += 1
            torch.cuda.synchronize()
            ep_loss = (acc / steps_per_epoch).cpu().numpy().tolist()
            history.append(ep_loss)
            log(f"  epoch {ep + 1}/{epochs}: train mse (scaled) {np.mean(ep_loss):.4f}, {time.time() - t0:.1f} s",
                flush=True)
    train_s = time.time() - t0
    _, m_te = evaluate(sur, X[te], T[te], batch)
    _, m_tr = evaluate(sur, X[tr[:te.numel()]], T[tr[:te.numel()]], batch)
    # the method without the learned part: a linear (Newtonian-like) map from
    # the current gradient alone, fitted by least squares on the training rows
    cur = X[:, 4 * (HIST - 1):4 * HIST].double()
    A = torch.cat([cur, torch.ones_like(cur[:, :1])], dim=1)
    coef = torch.linalg.lstsq(A[tr].cpu(), T[tr].double().cpu()).solution.to(dev)
    lin = (A[te] @ coef)
    lin_rel = float((lin - T[te].double()).norm() / T[te].double().norm())
    metrics = {"train_seconds": train_s, "steps": k, "epochs": epochs, "batch": batch, "lr": lr, "augment": augment,
               "train_rows": int(tr.numel()), "held_out_rows": int(te.numel()), "held_out": m_te,
               "train_subset": m_tr, "linear_current_gradient_rel_l2": lin_rel, "epoch_loss": history}
    return sur, metrics


def write_summary(metrics, path, command):
    """Markdown summary of a training run (data, training, errors)."""
    d, h = metrics["data"], metrics["held_out"]
    L = ["# Surrogate training: 5-member MLP ensemble 129-256-256-3 (BF16 matrix cores)", "",
         "Command (MI355X, one GPU):", "", "```", command, "```", "",
         "## Data generation (batched micro-DPD on the GPU)", "", "| quantity | value |", "|---|---|"]
    for k in ("n_boxes", "n_macro", "k_micro", "equil", "samples", "resets", "bad_samples", "grad_sd_range",
              "corr_steps_range", "shear"):
        L.append(f"| {k} | {d.get(k)} |")
    steps = d["n_macro"] * d["k_micro"] + d["equil"]
    L += [f"| wall time (s) | {d['seconds']:.1f} |",
          f"| particle-steps/s | {d['n_boxes'] * 4000 * steps / d['seconds']:.3e} |", "",
          "## Training", "", "| quantity | value |", "|---|---|"]
    for k in ("steps", "epochs", "batch", "lr", "augment", "train_rows", "held_out_rows"):
        L.append(f"| {k} | {metrics[k]} |")
    L += [f"| wall time (s) | {metrics['train_seconds']:.2f} |",
          f"| ms per Adam step (all members, with row gather) | {1000 * metrics['train_seconds'] / metrics['steps']:.3f} |",
          "", "## Errors (relative L2 over samples and the three outputs)", "", "| comparison | rel. L2 |", "|---|---|",
          f"| ensemble mean vs single DPD target, held-out boxes | {h['rel_l2']:.4f} |",
          f"| ensemble mean vs single DPD target, training boxes | {metrics['train_subset']['rel_l2']:.4f} |",
          f"| linear map of the current gradient only vs single target, held-out | "
          f"{metrics['linear_current_gradient_rel_l2']:.4f} |"]
    r = metrics.get("replicas")
    if r:
        R = r["info"]["replicas"]
        floor = r["dpd_single_noise_rel_l2"] / math.sqrt(R)
        model = math.sqrt(max(0.0, r["model_vs_replica_mean_rel_l2"] ** 2 - floor ** 2))
        L += [f"| DPD noise of one target ({R} replicas, same start and gradients) | {r['dpd_single_noise_rel_l2']:.4f} |",
              f"| ensemble mean vs {R}-replica mean (unseen seeds) | {r['model_vs_replica_mean_rel_l2']:.4f} |",
              f"| noise left in a {R}-replica mean | {floor:.4f} |",
              f"| model error with that noise removed in quadrature | {model:.4f} |"]
    L += ["", f"Mean ensemble spread (scaled units, targets / {STRESS_SCALE}): {h['mean_spread_scaled']:.4f}; "
          f"target RMS (scaled) {h['rmse_scaled'] / h['rel_l2']:.3f}.", "",
          "Train MSE (scaled) per epoch, mean over members: " +
          ", ".join(f"{sum(e) / len(e):.4f}" for e in metrics["epoch_loss"])]
    with open(path, "w") as f:
        f.write("\n".join(L) + "\n")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--boxes", type=int, default=4096)
    ap.add_argument("--macro", type=int, default=520)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--no-augment", action="store_true")
    ap.add_argument("--replica-groups", type=int, default=32)
    ap.add_argument("--replicas", type=int, default=8)
    ap.add_argument("--summary", default=None, help="also write a markdown summary here")
    ap.add_argument("--amp-range", default=f"{AMP_RANGE[0]},{AMP_RANGE[1]}",
                    help="range of u in the per-box gradient amplitude GRAD_SD x 10^u")
    ap.add_argument("--corr-range", default=f"{CORR_STEPS},{CORR_STEPS}",
                    help="range of the per-box gradient correlation time in macro steps (log-uniform)")
    ap.add_argument("--shear", default=None,
                    help="frac,lo,hi: that fraction of the boxes also gets a simple-shear OU of amplitude "
                         "GRAD_SD x 10^u, u in [lo, hi]")
    args = ap.parse_args(argv)
    import torch

    if not torch.cuda.is_available():
        raise SystemExit("the training pipeline runs on the GPU")
    os.makedirs(args.out, exist_ok=True)
    print(f"generating: {args.boxes} boxes x {args.macro} macro steps", flush=True)
    amp = tuple(float(v) for v in args.amp_range.split(","))
    corr = tuple(float(v) for v in args.corr_range.split(","))
    shear = tuple(float(v) for v in args.shear.split(",")) if args.shear else None
    X, T, box_id, step_id, info = generate(args.boxes, args.macro, amp_range=amp, corr_range=corr, shear=shear)
    print(json.dumps(info), flush=True)
    sur, metrics = train(X, T, box_id, epochs=args.epochs, augment=not args.no_augment)
    metrics["data"] = info
    print(json.dumps({k: v for k, v in metrics.items() if k != "epoch_loss"}), flush=True)
    del X, T
    if args.replica_groups > 0:
        nb = args.replica_groups * args.replicas
        print(f"replicas: {args.replica_groups} groups x {args.replicas}", flush=True)
        Xr, Tr, br, sr, rinfo = generate(nb, min(args.macro, 200), seed_k=5, replicas=args.replicas, amp_range=amp,
                                         corr_range=corr, shear=shear)
        M, _ = evaluate(sur, Xr, Tr, 4096)
        grp = (br // args.replicas).long() * 1000000 + sr.long()
        uniq, inv, counts = torch.unique(grp, return_inverse=True, return_counts=True)
        full = counts[inv] == args.replicas
        Tm = torch.zeros((uniq.numel(), 3), dtype=torch.float64, device=Tr.device).index_add_(0, inv, Tr.double())
        Tm = Tm / counts[:, None].double()
        dev_single = (Tr.double() - Tm[inv])[full]
        noise = float(dev_single.norm() / Tm[inv][full].norm()) * math.sqrt(args.replicas / (args.replicas - 1.0))
        model_vs_mean = float((M.double() - Tm[inv])[full].norm() / Tm[inv][full].norm())
        model_vs_single = float((M.double() - Tr.double())[full].norm() / Tr.double()[full].norm())
        metrics["replicas"] = {"info": rinfo, "dpd_single_noise_rel_l2": noise,
                               "model_vs_replica_mean_rel_l2": model_vs_mean,
                               "model_vs_single_rel_l2": model_vs_single}
        print(json.dumps(metrics["replicas"]), flush=True)
    W = sur.get_weights()
    arrays = {f"m{e}_{k}": W[e][k] for e in range(len(W)) for k in surrogate.LAYERS}
    np.savez(os.path.join(args.out, "surrogate.npz"), grad_scale=GRAD_SCALE, stress_scale=STRESS_SCALE,
             n_hidden=256, n_members=len(W), **arrays)
    with open(os.path.join(args.out, "train_metrics.json"), "w") as f:
        json.dump(metrics, f, indent=1)
    if args.summary:
        import sys

        write_summary(metrics, args.summary, "python -m paper_2512_13267_amd.train " + " ".join(sys.argv[1:]))
    print("done", flush=True)


if __name__ == "__main__":
    main()
