"""Benchmark: r-RESPA MD steps/s and three-body triplets/s on one MI355X.

One bench "step" is one r-RESPA outer cycle (Sec. 4.1, Algorithm 2): k inner steps,
each with cell binning, Lennard-Jones forces and the velocity-Verlet updates, plus one
Axilrod-Teller-Muto evaluation with its kicks and the energy reductions of that full
step.  The timed region is a single respa_step call of steps * k inner steps on inputs
already resident in HBM.

Default workload: 32,000 particles (20^3 FCC cells, rho 0.8, T 0.7, jitter 0.05), LJ
eps = sigma = 1 with rc 2.5, ATM nu = 0.073 with rc3 2.5, dt 0.001, k = 10, FP64.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "3-body triplets/s + r-RESPA MD steps/s, FP32 vs FP64 GPU at stated force error"
# Algorithmic work per in-cutoff ATM triplet (edge, ATM arithmetic, three forces and their
# accumulation; FMA = 2), and the published MI355X vector peaks.
FLOPS_PER_TRIPLET = 100.0
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}


def _workload(name: str):
    from paper_2507_11172_amd import workloads as W
    if name == "fcc32k":
        return W.fp64_at_scale()
    if name == "fcc500":
        return W.plain_fp64()
    if name == "fcc1m":
        return W.precision_form(10)
    raise SystemExit("unknown workload %s" % name)


def _params(w, precision: str, k: int):
    from paper_2507_11172_amd import mts
    return mts.Params(epsilon=w.epsilon, sigma=w.sigma, rc_pair=w.rc_pair, nu=w.nu,
                      rc_triplet=w.rc_triplet, mass=w.mass, dt=w.dt, k=k, precision=precision)


def run_gpu(w, precision: str, k: int, steps: int, warmup: int):
    import numpy as np
    import torch
    from paper_2507_11172_amd import mts

    dev = torch.device("cuda:0")
    sysm = mts.System(_params(w, precision, k), w.n_particles.tolist(), w.box)
    x = torch.tensor(w.x, dtype=torch.float64, device=dev)
    v = torch.tensor(w.v, dtype=torch.float64, device=dev)
    if warmup > 0:
        sysm.respa_step(x, v, warmup * k)
    sysm.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e = torch.zeros((steps + 1, w.n_systems, mts.MTS_NE), dtype=torch.float64, device=dev)
    sysm.respa_step(x, v, steps * k, e)
    sysm.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # live per-launch HIP-event timing of the force kernels, on the handle's stream
    sysm.enable_kernel_timing(True)
    sysm.respa_step(x, v, max(2, min(steps, 20)) * k)
    times = sysm.kernel_times()
    sysm.enable_kernel_timing(False)
    n_trip = sysm.count_triplets(x)
    sysm.sync()
    en = e.cpu().numpy()[:, 0, :]
    tot = en[:, 0] + en[:, 1] + en[:, 2]
    sysm.close()
    trip_launches, trip_ms = times["triplet"]
    pair_launches, pair_ms = times["pair"]
    return {
        "elapsed_s": elapsed,
        "inner_steps": steps * k,
        "triplets_per_eval": n_trip,
        "triplet_kernel_ms": trip_ms / max(trip_launches, 1),
        "pair_kernel_ms": pair_ms / max(pair_launches, 1),
        "triplet_launches": trip_launches,
        "pair_launches": pair_launches,
        "energy_drift_per_particle": float(abs(tot[-1] - tot[0]) / w.n_total),
        "rvite": float(np.mean(np.abs(tot - tot.mean())) / np.mean(en[:, 0])),
    }


def cpu_baseline(w, k: int):
    """The FP64 oracle as it stands, timed on this host: one pair and one triplet force
    evaluation of the whole system, scaled to inner steps/s for step-size factor k."""
    import oracle
    nthreads = oracle.num_threads()
    box = w.box[0]
    t0 = time.perf_counter()
    oracle.pair_forces(w.x, box, rc=w.rc_pair, nthreads=nthreads)
    t_pair = time.perf_counter() - t0
    t0 = time.perf_counter()
    r3 = oracle.triplet_forces(w.x, box, rc=w.rc_triplet, nthreads=nthreads)
    t_trip = time.perf_counter() - t0
    steps_per_s = k / (k * t_pair + t_trip)
    return {"value": steps_per_s, "unit": "MD steps/s", "cores": nthreads, "kind": "oracle",
            "sample": "one LJ pair evaluation (%.2f s) and one ATM triplet evaluation "
                      "(%.2f s, %d triplets) of the full %d-particle system, combined as "
                      "k=%d pair + 1 triplet evaluations per k inner steps"
                      % (t_pair, t_trip, r3.count, w.n_total, k),
            "triplets_per_s": r3.count / t_trip}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed r-RESPA outer cycles")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="fcc32k")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--k", type=int, default=0, help="override the step-size factor")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-form", action="store_true")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        return 2

    w = _workload(args.workload)
    k = args.k or w.k
    r = run_gpu(w, args.precision, k, args.steps, args.warmup)
    steps_per_s = r["inner_steps"] / r["elapsed_s"]
    ms_per_cycle = 1e3 * r["elapsed_s"] / args.steps
    trip_s = r["triplet_kernel_ms"] * 1e-3
    achieved = FLOPS_PER_TRIPLET * r["triplets_per_eval"] / trip_s / 1e12 if trip_s > 0 else 0.0
    peak = PEAK_TFLOPS[args.precision]
    out = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "MD steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_cycle,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_particles": w.n_total, "k": k,
                   "inner_steps": r["inner_steps"], "precision": args.precision,
                   "rc_pair": w.rc_pair, "rc_triplet": w.rc_triplet, "nu": w.nu, "dt": w.dt,
                   "step": "one r-RESPA outer cycle (k inner steps + 1 triplet evaluation)"},
        "triplets_per_s": r["triplets_per_eval"] / trip_s if trip_s > 0 else None,
        "triplets_per_eval": r["triplets_per_eval"],
        "kernel_ms": {"triplet": r["triplet_kernel_ms"], "pair": r["pair_kernel_ms"]},
        "energy_drift_per_particle": r["energy_drift_per_particle"],
        "rvite": r["rvite"],
        "roofline": {"bound": "alu", "kernel": "k_triplet", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None},
    }
    if not args.no_fp32_form and args.precision == "fp64":
        r32 = run_gpu(w, "fp32", k, args.steps, args.warmup)
        t32 = r32["triplet_kernel_ms"] * 1e-3
        out["fp32_form"] = {
            "value": r32["inner_steps"] / r32["elapsed_s"], "unit": "MD steps/s",
            "triplets_per_s": r32["triplets_per_eval"] / t32 if t32 > 0 else None,
            "kernel_ms": {"triplet": r32["triplet_kernel_ms"], "pair": r32["pair_kernel_ms"]},
            "roofline_frac_fp32_peak": (FLOPS_PER_TRIPLET * r32["triplets_per_eval"] / t32 / 1e12
                                        / PEAK_TFLOPS["fp32"]) if t32 > 0 else None,
            "energy_drift_per_particle": r32["energy_drift_per_particle"],
            "rvite": r32["rvite"],
        }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, k)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
