"""Benchmark of the batched micro-DPD step on one MI355X.

Workload: the 256-box batch (edges ~U(8, 16) rc at density 3, i.e. 1.5k-12k
particles per box, ~1.47M particles in total; polymer fraction ~U(0.1, 0.3)
in 10-bead FENE chains; a constant in-plane traceless gradient per box with
entries ~U(-0.5, 0.5)); single-precision particle state and pair forces,
double-precision cells and stress sums.  A step is one velocity-Verlet step
of every box (cell update, kick/drift, binning, pair + bond forces, kick,
stress).  Untimed set-up: 500 steps at rest relax the random start, the
relaxed state is kept on the device, the timed call's graph is captured and
replayed as warm-up, and the relaxed state is restored.  The timed region is
then one engine call of K steps (HIP-graph replays) on device-resident
state, the batch's first K steps under its gradients; the metric is
unordered DPD pairs within the cutoff evaluated per second (counted by the
engine itself).

Secondary legs (same JSON line): the coupled reverse-Poiseuille LHMM run
(plain batched DPD, macro steps/s) and the flow past a periodic array of
cylinders run twice, with all-DPD micro-domains and with the surrogate in
the loop (gate and DPD fallback): macro steps/s of each, the speed-up, the
fallback rate and the relative L2 error of the time-averaged deviatoric
stress of the surrogate run against the all-DPD run.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X (gfx950) published peaks: FP32 vector 157.3 TFLOP/s (256 CUs at
# 2.4 GHz, FMA counted as two flops, packed dual-issue); HBM3E 8 TB/s.
FP32_PEAK = 157.3e12
HBM_PEAK = 8.0e12  # bytes/s
# Algorithmic FP32 flops of one unordered pair within the cutoff (FMA = 2):
# image displacement 10, r^2 5, w and e 5, relative velocity with the
# streaming difference L d 12, e . v 5, force magnitude 8, the two force
# updates 9, virial 12, Box-Muller 6; the square root, reciprocal square
# root, log and cos and the Philox4x32-10 block (integer) are not flops.
PAIR_FLOPS = 73.0
# A finer cost model of the same unit: VALU lane-cycles of the method's own
# arithmetic per pair, Philox4x32-10 (10 rounds x (2 quarter-rate
# 32x32->64-bit multiplies + 2 three-input xors) = 100), Box-Muller (3
# quarter-rate transcendentals + 8 = 20), geometry (15), relative velocity
# (10), force and its two updates (13), virial (6), against the chip's
# 256 x 4 SIMD x 16 lanes x 2.4 GHz non-packed lane-cycle rate.
PAIR_LANE_CYCLES = 164.0
VALU_LANE_CYCLES_PEAK = 256 * 4 * 16 * 2.4e9


def measured_traffic(kernel_file: str, record: str):
    """HBM bytes per launch from a committed profiler record, or None when the
    kernel source has changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", record)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    sha = hashlib.sha256(open(os.path.join(ROOT, kernel_file), "rb").read()).hexdigest()
    return rec["hbm_bytes_per_launch"] if rec.get("source_sha256") == sha else None


def cpu_baseline(wl, budget_s: float = 12.0):
    """Time the FP64 oracle on a bounded sample of the same workload."""
    import oracle

    p = wl.params
    sample = list(range(16))
    boxes = [oracle.OracleBox(s=wl.boxes[k].s, c=wl.boxes[k].c, h=wl.boxes[k].h, n_chains=wl.boxes[k].n_chains,
                              box_id=k) for k in sample]
    Ls = [wl.boxes[k].L for k in sample]
    oracle.run_batch(p, p["seed"], p["chain_len"], boxes, Ls, 2)  # forces at the start, page-in
    pairs, steps, t0 = 0, 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        _, _, npairs = oracle.run_batch(p, p["seed"], p["chain_len"], boxes, Ls, 10, count_pairs=True)
        pairs += int(npairs.sum())
        steps += 10
    dt = time.perf_counter() - t0
    return {"value": pairs / dt, "unit": "pair-updates/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"boxes 0-15 of the 256-box batch ({sum(b.N for b in wl.boxes[:16])} particles), "
                      f"{steps} FP64 steps, {dt:.1f} s"}


def bench_lhmm(macro_steps: int, k_micro: int = 50, equil_steps: int = 500, warmup: int = 5):
    """Reverse-Poiseuille LHMM: 1024 SPH particles (16 x 64, quintic kernel of
    support 3 dh, dt 1e-3), one 4000-particle FP32 micro-box per particle
    (40 chains of 10 beads), k_micro micro steps per macro step.  The micro
    boxes first equilibrate equil_steps at zero gradient (untimed)."""
    import torch

    from paper_2512_13267_amd import inputs, lhmm, micro

    mac = inputs.reverse_poiseuille(n_steps=macro_steps)
    wl = inputs.lhmm_boxes(mac.n, n_particles=4000, seed_k=2)
    m = micro.from_workload(wl, precision="fp32")
    zero = torch.zeros((mac.n, 9), dtype=torch.float64, device="cuda")
    m.step(zero, equil_steps)
    s = lhmm.Sph(mac.params, mac.r, mac.v)
    cp = lhmm.Coupled(s, m)
    for _ in range(warmup):
        cp.step(k_micro)
    torch.cuda.synchronize()
    p0 = int(m.pair_total().sum())
    t0 = time.perf_counter()
    for _ in range(macro_steps):
        cp.step(k_micro)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    pairs = float(int(m.pair_total().sum()) - p0)  # every micro step of every timed interval
    flags = m.flags()
    r, v, d = s.get_state()
    out = {"metric": "LHMM macro steps/s (plain batched DPD)", "value": macro_steps / el,
           "ms_per_macro_step": el / macro_steps * 1e3, "macro_steps": macro_steps, "warmup": warmup,
           "workload": "reverse Poiseuille, 1024 SPH particles, 1024 micro-boxes x 4000 particles, "
                       f"{k_micro} micro steps per macro step", "micro_pair_updates_per_s": pairs / el,
           "micro_fp32_frac": PAIR_FLOPS * pairs / el / FP32_PEAK,
           "max_vx": float(np.abs(v[:, 0]).max()),
           "flagged_boxes": {"bond": int(np.count_nonzero(flags & 1)), "cell": int(np.count_nonzero(flags & 2))}}
    m.close()
    s.close()
    return out


def bench_pac(macro_steps: int, windows):
    """Cylinder-array LHMM (64 x 64 SPH lattice, ~3.6k micro-domains of 4000
    particles): all-DPD versus surrogate in the loop, same seeds; the stress
    error over each averaging window (the last macro steps)."""
    import torch

    from paper_2512_13267_amd import pac

    windows = sorted({min(int(w), macro_steps) for w in windows})
    out = {"workload": "flow past a periodic square array of cylinders (radius 0.2), 64 x 64 SPH lattice, "
                       "one 4000-particle micro-domain per mobile particle, 50 micro steps per macro step",
           "macro_steps": macro_steps, "avg_windows": windows, "gate_threshold": pac.GATE_THRESHOLD,
           "gate_floor": pac.GATE_FLOOR, "gate_max_grad": pac.gate_max_grad(), "gate_input_quantile": pac.GATE_INPUT_Q,
           "hold": pac.HOLD, "replay": pac.REPLAY}
    means = {}
    for mode in ("dpd", "surrogate"):
        ctx = pac.build(mode)
        r, means[mode] = pac.run(ctx, macro_steps, windows, log=lambda *a, **k: print(*a, file=sys.stderr, **k),
                                 label=mode)
        out["n_mobile"] = ctx["nm"]
        pac.close(ctx)
        torch.cuda.synchronize()
        out[mode] = {"macro_steps_per_s": r["macro_steps_per_s"], "fallback_rate": r["fallback_rate"],
                     "out_of_range_rate": r["out_of_range_rate"], "micro_box_steps": r["micro_box_steps"],
                     "resets": r["resets"], "entered": r["entered"]}
    out["speedup"] = out["surrogate"]["macro_steps_per_s"] / out["dpd"]["macro_steps_per_s"]
    out["stress_rel_l2_vs_dpd"] = {str(w): pac.compare(means["surrogate"][w], means["dpd"][w], out["n_mobile"])
                                   for w in windows}
    return out


def bench_surrogate(steps: int = 50):
    """Training step (5 members 129-256-256-3, batch 4096, the training
    configuration) and in-loop inference (3572 rows), timed with device
    synchronisation; matrix-core rate against the BF16 dense peak."""
    import torch

    from paper_2512_13267_amd import surrogate

    E, nin, nh, nout, B = 5, 129, 256, 3, 4096
    s = surrogate.Surrogate(surrogate.init_members(E, nin, nh, nout, seed=1), nin, nh, nout, max_batch=B)
    g = torch.Generator(device="cpu")
    g.manual_seed(7)
    X = torch.randn((B, nin), generator=g).cuda()
    T = torch.randn((B, nout), generator=g).cuda()
    for _ in range(5):
        s.train_step(X, T, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.train_step(X, T, 1e-4)
    torch.cuda.synchronize()
    train_ms = (time.perf_counter() - t0) / steps * 1e3
    Xi = X[:3572].contiguous()
    Y = s.forward(Xi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.forward(Xi, out=Y)
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t0) / steps * 1e3
    s.close()
    kp, hp = 160, nh  # padded input width, hidden width; outputs padded to 32
    fwd_flops = lambda b: 2.0 * E * b * (kp * hp + hp * hp + hp * 32)
    train_flops = fwd_flops(B) + 2.0 * E * B * (hp * 32 * 2 + hp * hp * 2 + kp * hp)
    peak = 2.5e15
    return {"train_step_ms": train_ms, "train_TFLOPs": train_flops / (train_ms * 1e-3) / 1e12,
            "train_mfma_frac": train_flops / (train_ms * 1e-3) / peak,
            "forward_3572_ms": fwd_ms, "forward_TFLOPs": fwd_flops(3584) / (fwd_ms * 1e-3) / 1e12,
            "peak_TFLOPs_bf16_dense": peak / 1e12,
            "shape": "5 members 129-256-256-3 (padded 160-256-256-32), batch 4096 train / 3572 inference"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--relax-steps", type=int, default=500,
                    help="untimed steps at rest from the random initial positions before the workload starts")
    ap.add_argument("--warmup-seconds", type=float, default=0.3,
                    help="the warm-up also lasts at least this long (in calls of the timed call's graph)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="search the launch parameters (lhmm_micro_autotune, cached) instead of keeping the engine's "
                         "defaults; its 20-step trials are noisier than the differences between the best configurations")
    ap.add_argument("--no-autotune", action="store_true", help="the default (kept for older command lines)")
    ap.add_argument("--timing-steps", type=int, default=None,
                    help="steps of the per-kernel timing (default: all the timed steps, from the same state)")
    ap.add_argument("--lhmm-steps", type=int, default=200,
                    help="macro steps of the coupled reverse-Poiseuille run (0 skips it)")
    ap.add_argument("--pac-steps", type=int, default=500,
                    help="macro steps of each cylinder-array run (all-DPD and surrogate; 0 skips them)")
    ap.add_argument("--pac-avg", default="100,400",
                    help="comma-separated averaging windows of the stress comparison (last macro steps)")
    ap.add_argument("--no-surrogate-timing", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 2^27 floats (512 MiB read, 512 MiB written) five "
                         "times, to scale the HBM byte counters of a profiler run")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch

        x = torch.ones(1 << 27, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": x.numel() * 4, "copy_calibration_bytes_written": y.numel() * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the micro-boxes are independent and "
              "would shard by box across GPUs, which is not implemented.", file=sys.stderr)
        sys.exit(2)
    if (args.steps < 1 or args.warmup < 0 or args.warmup_seconds < 0 or args.relax_steps < 0
            or (args.timing_steps is not None and args.timing_steps < 1)):
        print("bench.py needs --steps >= 1, --warmup >= 0, --warmup-seconds >= 0, --relax-steps >= 0 and "
              "--timing-steps >= 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2512_13267_amd import inputs, micro

    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    wl = inputs.batch()
    n_particles = wl.n_particles
    print(f"[bench] workload: {len(wl.boxes)} boxes, {n_particles} particles "
          f"(setup {time.perf_counter() - t_setup:.1f} s)", file=sys.stderr, flush=True)
    m = micro.from_workload(wl, precision="fp32")
    G = torch.tensor(np.stack([b.L for b in wl.boxes]), dtype=torch.float64, device="cuda").contiguous()

    # Set-up, untimed: the random initial positions (overlapping soft
    # spheres) relax at rest, as a micro-domain does before it is coupled.
    # The workload is then the first --steps steps under the gradients from
    # that relaxed state (forces included), kept on the device; the
    # warm-up, the timed call and the per-kernel timing all start from it.
    all_boxes = np.arange(len(wl.boxes), dtype=np.int32)
    if args.relax_steps > 0:
        m.step(torch.zeros_like(G), args.relax_steps)
    m.snapshot()
    torch.cuda.synchronize()
    print(f"[bench] relaxed {args.relax_steps} steps at rest", file=sys.stderr, flush=True)

    tuning = None
    if args.autotune and not args.no_autotune:
        from paper_2512_13267_amd import autotune

        tuning = autotune.tune(m, G, [b.N for b in wl.boxes], "fp32")
        print(f"[bench] launch parameters {tuning['config']} (cached: {tuning['cached']})", file=sys.stderr,
              flush=True)
        m.restore(all_boxes)
    # The warm-up replays the timed call's own graph (captured here, outside
    # the clock) until it has run at least --warmup steps and at least
    # --warmup-seconds: from idle the GPU needs some tens of milliseconds of
    # load to reach its working clock, so a few steps alone leave a short
    # timed call measuring the ramp rather than the kernels.
    m.prepare(args.steps)
    torch.cuda.synchronize()
    warm_steps, tw = 0, time.perf_counter()
    while warm_steps < args.warmup or time.perf_counter() - tw < args.warmup_seconds:
        m.step(G, args.steps)
        torch.cuda.synchronize()
        warm_steps += args.steps
    warm_s = time.perf_counter() - tw
    print(f"[bench] warmup done: {warm_steps} steps in {warm_s:.3f} s", file=sys.stderr, flush=True)
    m.restore(all_boxes)
    torch.cuda.synchronize()
    p0 = int(m.pair_total().sum())
    t0 = time.perf_counter()
    m.step(G, args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pairs = int(m.pair_total().sum()) - p0
    flags = m.flags()
    print(f"[bench] timed {args.steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)

    # per-kernel durations over the same steps from the same initial state,
    # grids and stream: eager launches with HIP events around each kernel
    timing_steps = args.steps if args.timing_steps is None else min(args.timing_steps, args.steps)
    m.restore(all_boxes)
    kt = m.time_kernels(G, timing_steps)
    pairs_timing = int(m.pair_counts().sum()) / timing_steps
    f_ms = kt["forces"]
    achieved = PAIR_FLOPS * pairs_timing / (f_ms * 1e-3)
    lane = PAIR_LANE_CYCLES * pairs_timing / (f_ms * 1e-3)
    traffic = measured_traffic("paper_2512_13267_amd/csrc/lhmm_micro.hip", "k_forces_batch256_traffic.json")
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": FP32_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": achieved / FP32_PEAK, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch", "kernel": "k_forces", "kernel_ms": f_ms, "timing_steps": timing_steps,
                "kernel_ms_all": kt, "pairs_per_launch": pairs_timing, "flops_per_pair": PAIR_FLOPS,
                "frac_of_nonpacked_fp32": achieved / (FP32_PEAK / 2),
                "method_lane_cycles": {"per_pair": PAIR_LANE_CYCLES, "achieved_T_per_s": lane / 1e12,
                                       "peak_T_per_s": VALU_LANE_CYCLES_PEAK / 1e12,
                                       "frac": lane / VALU_LANE_CYCLES_PEAK},
                "hbm_GBps": (traffic / (f_ms * 1e-3) / 1e9) if traffic else None,
                "hbm_frac": (traffic / (f_ms * 1e-3) / HBM_PEAK) if traffic else None}

    rec = {
        "metric": "micro-DPD pair-force updates/s",
        "value": pairs / elapsed,
        "unit": "pair-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warmup_run": {"steps": warm_steps, "seconds": warm_s},
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "256 DPD/FENE micro-boxes, edge U(8,16) rc, density 3, polymer fraction "
                               "U(0.1,0.3) in 10-bead chains, random positions relaxed at rest (untimed), then "
                               "constant planar gradients U(-0.5,0.5), FP32 forces / FP64 stress",
                   "relax_steps": args.relax_steps,
                   "n_boxes": len(wl.boxes), "n_particles": n_particles,
                   "pairs_per_step": pairs / args.steps,
                   "launch": m.config(), "tuned": tuning is not None,
                   "flagged_boxes": {"bond": int(np.count_nonzero(flags & 1)), "cell": int(np.count_nonzero(flags & 2)),
                                     "nonfinite": int(np.count_nonzero(flags & 4))}},
        "roofline": roofline,
    }
    m.close()
    if args.lhmm_steps > 0:
        print("[bench] coupled LHMM run", file=sys.stderr, flush=True)
        rec["lhmm"] = bench_lhmm(args.lhmm_steps)
        print(f"[bench] {rec['lhmm']['value']:.2f} macro steps/s", file=sys.stderr, flush=True)
    if not args.no_surrogate_timing:
        print("[bench] surrogate training and inference timing", file=sys.stderr, flush=True)
        rec["surrogate"] = bench_surrogate()
    if args.pac_steps > 0:
        print("[bench] cylinder-array LHMM: all-DPD and surrogate", file=sys.stderr, flush=True)
        rec["lhmm_pac"] = bench_pac(args.pac_steps, [int(w) for w in args.pac_avg.split(",")])
        print(f"[bench] surrogate {rec['lhmm_pac']['surrogate']['macro_steps_per_s']:.2f} vs DPD "
              f"{rec['lhmm_pac']['dpd']['macro_steps_per_s']:.2f} macro steps/s", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(wl)
    torch.cuda.synchronize()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
