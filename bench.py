"""Benchmark: r-RESPA MD steps/s and three-body triplets/s on one MI355X.

One bench "step" is one r-RESPA outer cycle (Sec. 4.1, Algorithm 2): k inner steps with
Lennard-Jones forces and the velocity-Verlet updates, plus one Axilrod-Teller-Muto
evaluation with its kicks and the energy reductions of that full step.  The timed region
is a single respa_step call of steps * k inner steps on inputs already resident in HBM.

Default workload: 1,048,576 particles (64^3 FCC cells, rho 0.8, T 0.7, jitter 0.05), LJ
eps = sigma = 1 with rc 2.5, ATM nu = 0.073 with rc3 2.5, dt 0.001, k = 10, FP64, with
the FP32 form and the CPU oracle (its exact subset mode on 4,000 seeded particles, scaled
to the whole system) timed beside it.  Other workloads (--workload):
  fcc32k   32,000 particles (20^3 FCC cells), k = 10, FP64 (--k to sweep)
  fcc500   500 particles, k = 1 (velocity Verlet), FP64
  slab25   500,000-particle liquid slab + vapour, 1:1:3 box, rc3 2.5, FP32 form, k = 10
  slab30   the same with rc3 3.0
  batched  256 replicas of 200..20,000 particles in one handle, FP32 form, k = 10, with
           the same replicas run one handle at a time for comparison
  toy675   DirectSum (every pair and triplet, open boundaries): the RVITE study's toy
           scenario, 675 particles in a 10^3 domain, nu 0.3, FP64, k = 1
  al4995   DirectSum: the aluminium scenario, 4,995 particles in a 20^3 domain,
           nu 0.3095, dt 0.00304, FP64, k = 12
Prints one JSON line.  For several systems "value" is the aggregate over systems
(system inner steps per second).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "3-body triplets/s + r-RESPA MD steps/s, FP32 vs FP64 GPU at stated force error"
# Algorithmic work per in-cutoff ATM triplet (edge, ATM arithmetic, three forces and their
# accumulation; FMA = 2), and the published MI355X vector peaks (the FP32 figure assumes
# packed FP32 instructions, which this library does not emit: its FP32 arithmetic runs at
# the unpacked rate, equal to the FP64 one).
FLOPS_PER_TRIPLET = 100.0
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}
# HBM bytes per launch of the triplet launch, measured by FETCH_SIZE and WRITE_SIZE
# counter runs of `bench.py --traffic-probe` and scaled by the counts of a 256 MiB copy;
# stored in profiles/hbm_traffic.json with a hash of the kernel's sources, so that a
# changed kernel reports null until its counters are taken again.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
TRIPLET_SOURCES = ("triplet.hip", "atm.h", "common.h", "list_build.h")
# Algorithmic bytes per particle of one list force launch (k_pair_list) besides its list
# row: own sorted position 32, perm and system index 8, row length 4, F2 written 24, and
# the fused update of a plain inner step: v read and written 48, previous F2 read 24, x
# read and written 48, skin reference read 24, drifted sorted position written 24.
PAIR_BYTES_FIXED = 256
PAIR_BYTES_PER_ENTRY = 4  # one int32 neighbour index per list entry
HBM_PEAK_GBS = 8000.0


def kernel_sources_sha(names=TRIPLET_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2507_11172_amd", "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def stored_traffic(workload: str, precision: str, kernel: str):
    """HBM bytes per launch from the committed counter summary, or None when no counter
    run covers this workload, precision and kernel at the current sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            rows = json.load(f)
    except (OSError, ValueError):
        return None
    sha = kernel_sources_sha()
    for r in rows:
        if (r.get("workload"), r.get("precision"), r.get("kernel_reported"),
                r.get("sources_sha")) == (workload, precision, kernel, sha):
            return r.get("bytes_per_launch")
    return None


def _workload(name: str):
    from paper_2507_11172_amd import workloads as W
    table = {
        "fcc32k": W.fp64_at_scale,
        "fcc500": W.plain_fp64,
        "fcc1m": lambda: W.precision_form(10),
        "fcc1m_fp32": lambda: W.precision_form(10, "fp32"),
        "slab25": lambda: W.inhomogeneous(2.5),
        "slab30": lambda: W.inhomogeneous(3.0),
        "batched": W.batched,
        "toy675": lambda: W.toy(nu=0.3),
        "al4995": W.aluminium,
        "fcc32k_nested": W.nested_at_scale,
    }
    if name not in table:
        raise SystemExit("unknown workload %s (one of %s)" % (name, ", ".join(table)))
    return table[name]()


def _params(w, precision: str, k: int):
    from paper_2507_11172_amd import mts
    return mts.Params(epsilon=w.epsilon, sigma=w.sigma, rc_pair=w.rc_pair, nu=w.nu,
                      rc_triplet=w.rc_triplet, mass=w.mass, dt=w.dt, k=k, precision=precision,
                      method=w.method, k_outer=w.k_outer, rc_triplet_inner=w.rc_triplet_inner)


def _drift_stats(en, n_particles):
    """Energy drift per particle and RVITE (Eq. 4) per system from the full-step records
    [rows][systems][K, U2, U3, W2, W3]; means over systems."""
    import numpy as np
    tot = en[:, :, 0] + en[:, :, 1] + en[:, :, 2]
    drift = np.abs(tot[-1] - tot[0]) / n_particles
    rvite = np.mean(np.abs(tot - tot.mean(axis=0)), axis=0) / np.mean(en[:, :, 0], axis=0)
    return float(drift.mean()), float(rvite.mean())


# Runs repeated after a capacity overflow: every overflow enlarges what overflowed (tile,
# lists), so the sizes grow monotonically; a batch of many systems can reveal a few in turn.
CAPACITY_ATTEMPTS = 8


def run_gpu(w, precision: str, k: int, steps: int, warmup: int, tune_ms: int):
    import numpy as np
    import torch
    from paper_2507_11172_amd import mts

    dev = torch.device("cuda:0")
    span = k * w.k_outer  # inner steps per full step
    sysm = mts.System(_params(w, precision, k), w.n_particles.tolist(), w.box)
    x = torch.tensor(w.x, dtype=torch.float64, device=dev)
    v = torch.tensor(w.v, dtype=torch.float64, device=dev)
    # one-time set-up outside the timed region, like the graph capture of the warm-up
    tuning = sysm.autotune(x, v, tune_ms) if tune_ms > 0 else sysm.tuning()
    x0, v0 = x.clone(), v.clone()
    for attempt in range(CAPACITY_ATTEMPTS):
        if warmup > 0:
            sysm.respa_step(x, v, warmup * span)
        try:
            sysm.sync()
            break
        except mts.MTSError as err:
            # a tile or list outgrew its initial size: the library has enlarged it, and
            # the warm-up is repeated from the initial state
            if err.code != mts.MTS_ERR_CAPACITY or attempt == CAPACITY_ATTEMPTS - 1:
                raise
            print(f"warm-up repeated: {err}", file=sys.stderr, flush=True)
            x.copy_(x0)
            v.copy_(v0)
    e = torch.zeros((steps + 1, w.n_systems, mts.MTS_NE), dtype=torch.float64, device=dev)
    x1, v1 = x.clone(), v.clone()
    for attempt in range(CAPACITY_ATTEMPTS):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sysm.respa_step(x, v, steps * span, e)
        try:
            sysm.sync()
        except mts.MTSError as err:
            # a list outgrew its size or a particle outran the skin: the library has
            # enlarged it; the timed run is repeated from the same state
            if err.code != mts.MTS_ERR_CAPACITY or attempt == CAPACITY_ATTEMPTS - 1:
                raise
            print(f"timed run repeated: {err}", file=sys.stderr, flush=True)
            x.copy_(x1)
            v.copy_(v1)
            continue
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        break

    # live per-launch HIP-event timing of the force kernels, on the handle's stream (with
    # the energy records, as in the timed region: the same kernel variants).  Every
    # respa_step call opens with one evaluation of the entry forces, so two calls of nt1
    # and nt2 cycles are timed and differenced: what remains is exactly nt2 - nt1 full
    # steps of the r-RESPA cycle.
    nt1 = 2
    nt2 = nt1 + max(2, min(steps, 20))
    sysm.enable_kernel_timing(True)
    passes = []
    for nt in (nt1, nt2):
        sysm.respa_step(x, v, nt * span, torch.zeros((nt + 1, w.n_systems, mts.MTS_NE),
                                                     dtype=torch.float64, device=dev))
        passes.append(sysm.kernel_times())
    sysm.enable_kernel_timing(False)
    nt = nt2 - nt1
    times = {c: (passes[1][c][0] - passes[0][c][0], passes[1][c][1] - passes[0][c][1])
             for c in ("triplet", "pair")}
    n_trip = sysm.count_triplets(x)
    sysm.sync()
    sysm.close()
    n_inner = 0
    if w.k_outer > 1:  # size of the inner distance class at the same positions
        import dataclasses
        wi = dataclasses.replace(w, rc_triplet=w.rc_triplet_inner, k_outer=1, rc_triplet_inner=0.0)
        with mts.System(_params(wi, precision, k), w.n_particles.tolist(), w.box) as si:
            n_inner = si.count_triplets(x)
    drift, rvite = _drift_stats(e.cpu().numpy(), w.n_particles)
    trip_launches, trip_ms = times["triplet"]
    pair_launches, pair_ms = times["pair"]
    skin = float(tuning.get("skin", 0.0))
    rv3 = (w.rc_pair + skin) ** 3
    list_entries = sum(float(n) * (float(n) / float(np.prod(b))) * 4.0 / 3.0 * math.pi * rv3
                       for n, b in zip(w.n_particles, w.box))
    return {
        "elapsed_s": elapsed,
        "list_entries_est": list_entries,
        "inner_steps": steps * span,
        "triplets_per_eval": n_trip,
        "inner_class_triplets": n_inner,
        "triplet_ms_per_full_step": trip_ms / nt,
        "triplet_launches_per_full_step": trip_launches / nt,
        "triplet_kernel_ms": trip_ms / max(trip_launches, 1),
        "pair_kernel_ms": pair_ms / max(pair_launches, 1),
        "energy_drift_per_particle": drift,
        "rvite": rvite,
        "tuning": tuning,
    }


def fp32_force_error(w, k: int):
    """The FP32 form's force and energy error against the FP64 path on the GPU, at the
    workload's initial state, each the largest over the systems: max |dF| / RMS |F| of a
    system for F2 and F3, and |dE| / N of a system's total potential energy."""
    import numpy as np
    import torch
    from paper_2507_11172_amd import mts

    dev = torch.device("cuda:0")
    out = {}
    for prec in ("fp64", "fp32"):
        with mts.System(_params(w, prec, k), w.n_particles.tolist(), w.box) as s:
            x = torch.tensor(w.x, dtype=torch.float64, device=dev)
            f2, f3 = torch.empty_like(x), torch.empty_like(x)
            e2 = torch.zeros((w.n_systems, 2), dtype=torch.float64, device=dev)
            e3 = torch.zeros((w.n_systems, 2), dtype=torch.float64, device=dev)
            s.compute_pair_forces(x, f2, e2)
            s.compute_triplet_forces(x, f3, e3)
            s.sync()
            out[prec] = (f2.cpu().numpy(), f3.cpu().numpy(),
                         (e2[:, 0] + e3[:, 0]).cpu().numpy())

    starts = np.concatenate([[0], np.cumsum(w.n_particles)])

    def rel(a, r):  # the largest per-system max |dF| / RMS |F|
        worst = 0.0
        for lo, hi in zip(starts[:-1], starts[1:]):
            ref = r[lo:hi]
            rms = np.sqrt(np.mean(np.sum(ref * ref, axis=1))) if hi > lo else 0.0
            if rms > 0:
                worst = max(worst, float(np.abs(a[lo:hi] - ref).max() / rms))
        return worst

    (a2, a3, ae), (b2, b3, be) = out["fp32"], out["fp64"]
    return {"f2": rel(a2, b2), "f3": rel(a3, b3),
            "energy_per_particle": float(np.max(np.abs(ae - be) / np.maximum(w.n_particles, 1))),
            "bars": "1e-5 on forces, 1e-7 per particle on energy"}


def run_per_system_loop(w, precision: str, k: int, steps: int):
    """The same replicas, one handle each, stepped one after another: aggregate system
    inner steps per second of that launch loop."""
    import torch
    from paper_2507_11172_amd import mts

    dev = torch.device("cuda:0")
    handles, xs, vs = [], [], []
    off = 0
    for r in range(w.n_systems):
        n = int(w.n_particles[r])
        handles.append(mts.System(_params(w, precision, k), [n], w.box[r:r + 1]))
        xs.append(torch.tensor(w.x[off:off + n], dtype=torch.float64, device=dev))
        vs.append(torch.tensor(w.v[off:off + n], dtype=torch.float64, device=dev))
        off += n
    for h, x, v in zip(handles, xs, vs):  # warm-up: graphs captured, caches sized
        for attempt in range(3):
            h.respa_step(x, v, k)
            try:
                h.sync()
                break
            except mts.MTSError as err:
                if err.code != mts.MTS_ERR_CAPACITY or attempt == 2:
                    raise
    x0 = [x.clone() for x in xs]
    v0 = [v.clone() for v in vs]
    for attempt in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for h, x, v in zip(handles, xs, vs):
            h.respa_step(x, v, steps * k)
        grown = False
        for h in handles:
            try:
                h.sync()
            except mts.MTSError as err:
                # a replica's list outgrew its size mid-run: enlarged, timed again
                if err.code != mts.MTS_ERR_CAPACITY or attempt == 2:
                    raise
                grown = True
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        if not grown:
            break
        for x, v, a, b in zip(xs, vs, x0, v0):
            x.copy_(a)
            v.copy_(b)
    for h in handles:
        h.close()
    return w.n_systems * steps * k / elapsed


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(w, k: int):
    """The FP64 oracle as it stands, timed on this host: one pair and one triplet force
    evaluation of the whole system, scaled to inner steps/s for step-size factor k."""
    import oracle
    nthreads = oracle.num_threads()
    if w.method == "direct":
        return _cpu_baseline_direct(w, k, nthreads)
    box = w.box[0]
    t0 = time.perf_counter()
    oracle.pair_forces(w.x, box, rc=w.rc_pair, nthreads=nthreads)
    t_pair = time.perf_counter() - t0
    t0 = time.perf_counter()
    r3 = oracle.triplet_forces(w.x, box, rc=w.rc_triplet, nthreads=nthreads)
    t_trip = time.perf_counter() - t0
    if w.k_outer > 1:
        # nested (the oracle's loop): per full step k * k_outer pair evaluations, the inner
        # class k_outer times and the outer class once (about the cost of the whole set)
        span = k * w.k_outer
        t0 = time.perf_counter()
        ri = oracle.triplet_forces(w.x, box, rc=w.rc_triplet_inner, nthreads=nthreads)
        t_in = time.perf_counter() - t0
        return {"value": span / (span * t_pair + w.k_outer * t_in + t_trip), "unit": "MD steps/s",
                "cores": nthreads, "kind": "oracle", "cpu": _cpu_model(),
                "sample": "one LJ evaluation (%.2f s), one evaluation of the inner class "
                          "(%.2f s, %d triplets) and one of the whole cutoff set (%.2f s, %d "
                          "triplets) of the %d-particle system, combined as %d pair + %d inner "
                          "+ 1 whole-set evaluations per full step of %d inner steps"
                          % (t_pair, t_in, ri.count, t_trip, r3.count, w.n_total, span,
                             w.k_outer, span),
                "triplets_per_s": (r3.count + ri.count) / (t_trip + t_in)}
    steps_per_s = k / (k * t_pair + t_trip)
    return {"value": steps_per_s, "unit": "MD steps/s", "cores": nthreads, "kind": "oracle",
            "cpu": _cpu_model(),
            "sample": "one LJ pair evaluation (%.2f s) and one ATM triplet evaluation "
                      "(%.2f s, %d triplets) of the full %d-particle system, combined as "
                      "k=%d pair + 1 triplet evaluations per k inner steps"
                      % (t_pair, t_trip, r3.count, w.n_total, k),
            "triplets_per_s": r3.count / t_trip}


SUBSET_SAMPLE = 4000  # particles of the oracle's exact subset mode on large systems
SUBSET_SAMPLE_SINGLE = 1000  # the same on one thread (a bounded run)


def cpu_baseline_subset(w, k: int):
    """The oracle's exact subset mode on seeded particles of a large system (every pair
    and triplet holding each sampled particle, found by a scan over all N): 4,000
    particles on all host cores, 1,000 on one.  Scaled to the whole system: one
    evaluation of both forces costs N / sample times the sample's.  A cycle of k inner
    steps needs k pair evaluations and one triplet evaluation; each pair evaluation costs
    the same O(N) scan per particle as the combined one (the triplet loop adds little),
    so a cycle is scaled as k combined evaluations.  Triplets/s: the sample's triplet
    visits / 3 (each triplet is visited from its three members) per second."""
    import numpy as np
    import oracle
    from paper_2507_11172_amd import workloads as W
    box = w.box[0]
    n = w.n_total
    out = {}
    for label, nthreads, m in (("all", oracle.num_threads(), SUBSET_SAMPLE),
                               ("single", 1, SUBSET_SAMPLE_SINGLE)):
        idx = np.sort(W.rng_for(78).choice(n, size=min(m, n), replace=False))
        t0 = time.perf_counter()
        _, _, (_, ntrip) = oracle.subset_forces(w.x, box, idx, rc_pair=w.rc_pair, nu=w.nu,
                                                rc3=w.rc_triplet, nthreads=nthreads, counts=True)
        t = time.perf_counter() - t0
        full = t * n / idx.shape[0]  # one whole-system evaluation of F2 and F3
        out[label] = {"value": k / (k * full), "triplets_per_s": ntrip / 3.0 / t,
                      "cores": nthreads, "sample_particles": int(idx.shape[0]),
                      "sample_s": t, "triplet_visits": ntrip}
    a, one = out["all"], out["single"]
    return {"value": a["value"], "unit": "MD steps/s", "cores": a["cores"], "kind": "oracle",
            "cpu": _cpu_model(), "scaled": True,
            "sample": "exact subset mode (scan of all N per particle, every pair and triplet "
                      "holding it) on %d seeded particles of the %d-particle system: %.2f s "
                      "on %d threads, %d triplet visits; scaled by N / %d to a whole-system "
                      "evaluation, and a cycle of k = %d inner steps as k such evaluations"
                      % (a["sample_particles"], n, a["sample_s"], a["cores"],
                         a["triplet_visits"], a["sample_particles"], k),
            "triplets_per_s": a["triplets_per_s"],
            "single_thread": {k2: one[k2] for k2 in ("value", "triplets_per_s", "cores",
                                                     "sample_particles", "sample_s")}}


def _cpu_baseline_direct(w, k: int, nthreads: int):
    """DirectSum through the oracle: a box far larger than the cluster and a cutoff beyond
    every distance.  The pair evaluation runs on the whole system; the O(N^3) triplet one on
    the first M particles, M chosen for a few seconds of work, its rate scaled to C(N, 3)."""
    import math
    import numpy as np
    import oracle
    big, rc = np.full(3, 1.0e6), 4.0e5
    x = w.x - w.x.min(axis=0) + 1.0
    n = x.shape[0]
    t0 = time.perf_counter()
    oracle.pair_forces(x, big, rc=rc, shift=False, nthreads=nthreads)
    t_pair = time.perf_counter() - t0
    m = min(n, 1200)
    t0 = time.perf_counter()
    r3 = oracle.triplet_forces(x[:m], big, nu=w.nu, rc=rc, nthreads=nthreads)
    t_m = time.perf_counter() - t0
    rate = r3.count / t_m
    t_trip = math.comb(n, 3) / rate
    return {"value": k / (k * t_pair + t_trip), "unit": "MD steps/s", "cores": nthreads,
            "kind": "oracle", "cpu": _cpu_model(),
            "sample": "DirectSum: one LJ evaluation of all %d particles (%.2f s) and one ATM "
                      "evaluation of the first %d (%.2f s, %d triplets), its rate scaled to "
                      "the C(N,3) = %d triplets of the system; k=%d pair + 1 triplet "
                      "evaluations per k inner steps" % (n, t_pair, m, t_m, r3.count,
                                                         math.comb(n, 3), k),
            "triplets_per_s": rate}


def rvite_sweep(nus, ks, n_iter: int, precision: str):
    """RVITE (Eq. 4) of the toy scenario (675 particles in a 10^3 domain, DirectSum, the
    same seeded initial state for every run) for each nu and step-size factor: n_iter inner
    steps of r-RESPA with energy records at every full step."""
    import numpy as np
    import torch
    from paper_2507_11172_amd import mts, workloads as W

    dev = torch.device("cuda:0")
    bad = [k for k in ks if n_iter % k]
    if bad:
        raise SystemExit("--sweep-iter %d is not a multiple of %s" % (n_iter, bad))
    table, seconds = {}, 0.0
    for nu in nus:
        w = W.toy(nu=nu)
        row = {}
        for k in ks:
            with mts.System(_params(w, precision, k), w.n_particles.tolist(), w.box) as s:
                x = torch.tensor(w.x, dtype=torch.float64, device=dev)
                v = torch.tensor(w.v, dtype=torch.float64, device=dev)
                e = torch.zeros((n_iter // k + 1, 1, mts.MTS_NE), dtype=torch.float64, device=dev)
                t0 = time.perf_counter()
                s.respa_step(x, v, n_iter, e)
                s.sync()
                seconds += time.perf_counter() - t0
            en = e.cpu().numpy()
            _, rv = _drift_stats(en, w.n_particles)
            row[str(k)] = rv
        table["%g" % nu] = row
        print("nu %g: %s" % (nu, " ".join("k%s=%.3e" % kv for kv in row.items())),
              file=sys.stderr, flush=True)
    # trend of RVITE with nu for each factor: slope of log(RVITE) against nu
    trend = {}
    for k in ks:
        y = np.log([table["%g" % nu][str(k)] for nu in nus])
        trend[str(k)] = float(np.polyfit(nus, y, 1)[0]) if len(nus) > 1 else 0.0
    return {"experiment": "RVITE vs nu and step-size factor, toy scenario (Sec. 4.2.1)",
            "method": "direct", "n_particles": 675, "box": 10.0, "dt": W.DT,
            "n_iter": n_iter, "precision": precision, "rvite": table,
            "dlogRVITE_dnu": trend, "gpu_seconds": seconds, "data": "synthetic"}


def nested_study(n_iter: int, nu: float, precision: str, schemes, workload: str = "fcc32k"):
    """Cost and accuracy of nested r-RESPA against plain step-size factors on a cutoff
    system (the 32,000-particle one, or the aluminium parameters in a periodic box with
    workload "al4995_pbc"; nu <= 0 keeps the workload's own): for each scheme (k, k_outer,
    r_a) the MD steps/s of one respa_step call of n_iter inner steps and the relative
    deviation of its total energy from Stoermer-Verlet's (k = 1) at the common full steps
    (the metric of Sec. 4.2.2, Fig. 4; both runs share the cutoff's own fluctuations)."""
    import dataclasses
    import numpy as np
    import torch
    from paper_2507_11172_amd import mts, workloads as W

    dev = torch.device("cuda:0")
    base = W.aluminium_periodic() if workload == "al4995_pbc" else W.fp64_at_scale()
    if nu > 0.0:
        base = dataclasses.replace(base, nu=nu)
    common = 1
    for k, ko, _ in schemes:
        common = common * (k * ko) // math.gcd(common, k * ko)
    if n_iter % common:
        raise SystemExit("--study-iter %d is not a multiple of %d" % (n_iter, common))
    runs = []
    for k, ko, ra in [(1, 1, 0.0)] + list(schemes):
        w = dataclasses.replace(base, k_outer=ko, rc_triplet_inner=ra)
        span = k * ko
        with mts.System(_params(w, precision, k), w.n_particles.tolist(), w.box) as s:
            x = torch.tensor(w.x, dtype=torch.float64, device=dev)
            v = torch.tensor(w.v, dtype=torch.float64, device=dev)
            s.respa_step(x.clone(), v.clone(), span)  # capture the graphs
            s.sync()
            e = torch.zeros((n_iter // span + 1, 1, mts.MTS_NE), dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.respa_step(x, v, n_iter, e)
            s.sync()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        en = e.cpu().numpy()[:, 0, :]
        tot = en[:, 0] + en[:, 1] + en[:, 2]
        runs.append({"k": k, "k_outer": ko, "rc_triplet_inner": ra, "steps_per_s": n_iter / dt,
                     "total": tot[:: common // span], "kinetic": en[:, 0]})
        print("scheme k=%d k_outer=%d r_a=%g: %.0f steps/s" % (k, ko, ra, n_iter / dt),
              file=sys.stderr, flush=True)
    ref = runs[0]["total"]
    out = []
    for r in runs:
        dev_rel = np.abs(r["total"] - ref) / np.abs(ref)
        out.append({"k": r["k"], "k_outer": r["k_outer"], "rc_triplet_inner": r["rc_triplet_inner"],
                    "steps_per_s": r["steps_per_s"],
                    "mean_rel_dev_vs_sv": float(dev_rel.mean()),
                    "max_rel_dev_vs_sv": float(dev_rel.max()),
                    "rvite": float(np.mean(np.abs(r["total"] - r["total"].mean()))
                                   / np.mean(r["kinetic"]))})
    return {"experiment": "nested r-RESPA over triplet distance classes vs plain step-size "
                          "factors (cost, and total-energy deviation from Stoermer-Verlet)",
            "workload": base.name, "n_particles": base.n_total, "nu": base.nu, "n_iter": n_iter,
            "precision": precision, "compare_every": common, "schemes": out,
            "data": "synthetic"}


def _run_chunked(s, x, v, n_iter: int, span: int, chunk: int, label: str, on_chunk=None):
    """respa_step in chunks of `chunk` inner steps (a resumed run equals one call); returns
    the energy records [n_iter / span + 1][systems][5]; prints one line per chunk."""
    import numpy as np
    import torch
    from paper_2507_11172_amd import mts
    rows = []
    done = 0
    while done < n_iter:
        m = min(chunk, n_iter - done)
        e = torch.zeros((m // span + 1, s.n_systems, mts.MTS_NE), dtype=torch.float64,
                        device=x.device)
        s.respa_step(x, v, m, e)
        s.sync()
        en = e.cpu().numpy()
        rows.append(en if not rows else en[1:])
        done += m
        if on_chunk is not None:
            on_chunk(x)
        print("%s: %d / %d inner steps" % (label, done, n_iter), file=sys.stderr, flush=True)
    return np.concatenate(rows, axis=0)


def al_energy_study(n_iter: int, ks, precision: str):
    """The aluminium scenario's total-energy deviation from Stoermer-Verlet (Sec. 4.2.2,
    Fig. 4) on DirectSum: one run per step-size factor from the same initial state, total
    energy at every 12th iteration (a full step of every factor), its relative deviation
    from the k = 1 run, binned into 50 bins over the range of all factors' deviations."""
    import numpy as np
    import torch
    from paper_2507_11172_amd import mts, workloads as W

    dev = torch.device("cuda:0")
    w = W.aluminium()
    common = 12
    if n_iter % common or any(common % k for k in ks):
        raise SystemExit("--al-iter must be a multiple of 12 and every factor divide 12")
    ks = [1] + [k for k in ks if k != 1]
    tot, seconds = {}, 0.0
    for k in ks:
        with mts.System(_params(w, precision, k), w.n_particles.tolist(), w.box) as s:
            x = torch.tensor(w.x, dtype=torch.float64, device=dev)
            v = torch.tensor(w.v, dtype=torch.float64, device=dev)
            t0 = time.perf_counter()
            en = _run_chunked(s, x, v, n_iter, k, 240, "aluminium DirectSum k=%d" % k)
            seconds += time.perf_counter() - t0
        t = en[:, 0, 0] + en[:, 0, 1] + en[:, 0, 2]
        tot[k] = t[:: common // k]
    ref = tot[1]
    rel = {k: (tot[k] - ref) / np.abs(ref) for k in ks}
    lo = min(float(rel[k].min()) for k in ks if k != 1)
    hi = max(float(rel[k].max()) for k in ks if k != 1)
    edges = np.linspace(lo, hi, 51) if hi > lo else np.linspace(lo - 1e-12, hi + 1e-12, 51)
    out = {}
    for k in ks:
        mean = float(tot[k].mean())
        h, _ = np.histogram(rel[k], bins=edges)
        out[str(k)] = {"mean_total_energy": mean,
                       "max_dev_from_mean_pct": float(100 * np.abs(tot[k] - mean).max() / abs(mean)),
                       "mean_rel_dev_vs_sv": float(rel[k].mean()),
                       "hist": (h / max(len(rel[k]), 1)).tolist()}
    return {"experiment": "aluminium total energy vs Stoermer-Verlet, DirectSum (Sec. 4.2.2, "
                          "Fig. 4)", "n_particles": w.n_total, "n_iter": n_iter, "dt": w.dt,
            "nu": w.nu, "precision": precision, "every": common,
            "bin_edges_rel_dev": edges.tolist(), "factors": out, "gpu_seconds": seconds,
            "data": "synthetic"}


def _rdf(x, box, r_max: float, nbins: int):
    """Pair counts of one frame in nbins shells up to r_max (minimum image)."""
    import numpy as np
    n = x.shape[0]
    counts = np.zeros(nbins)
    for i0 in range(0, n, 512):
        d = x[i0:i0 + 512, None, :] - x[None, :, :]
        d -= box * np.rint(d / box)
        r = np.sqrt(np.sum(d * d, axis=-1))
        ii = np.arange(i0, min(n, i0 + 512))[:, None]
        jj = np.arange(n)[None, :]
        counts += np.histogram(r[jj > ii], bins=nbins, range=(0.0, r_max))[0]
    return counts


def al_pbc_study(n_iter: int, n_eq: int, ks, precision: str):
    """The aluminium parameters on the cutoff path with periodic boundaries (Sec. 4.2.2,
    Figs. 6 and 7): after n_eq Stoermer-Verlet steps, one run of n_iter steps per
    step-size factor and one pure two-body run (nu = 0), all from the equilibrated state.
    Pressure (2K + W2 + W3) / 3V at every full step, binned into 20 bins over the range of
    all runs; radial distribution function from ten frames per run (host-side analysis of
    positions copied back)."""
    import dataclasses
    import math as m
    import numpy as np
    import torch
    from paper_2507_11172_amd import mts, workloads as W

    dev = torch.device("cuda:0")
    w = W.aluminium_periodic()
    box = w.box[0]
    vol = float(np.prod(box))
    x = torch.tensor(w.x, dtype=torch.float64, device=dev)
    v = torch.tensor(w.v, dtype=torch.float64, device=dev)
    with mts.System(_params(w, precision, 1), w.n_particles.tolist(), w.box) as s:
        _run_chunked(s, x, v, n_eq, 1, max(n_eq // 4, 12), "aluminium PBC equilibration")
    x_eq, v_eq = x.clone(), v.clone()
    r_max, nbins = 5.0, 100
    runs = [("two-body", 1, 0.0)] + [("k=%d" % k, k, w.nu) for k in ks]
    chunk = n_iter // 10
    if n_iter % 10 or any(chunk % k for _, k, _ in runs):
        raise SystemExit("--al-pbc-iter / 10 must be a multiple of every factor")
    res = {}
    for label, k, nu in runs:
        wk = dataclasses.replace(w, nu=nu)
        x, v = x_eq.clone(), v_eq.clone()
        acc = np.zeros(nbins)
        frames = [0]

        def frame(xd):
            acc[:] += _rdf(xd.cpu().numpy(), box, r_max, nbins)
            frames[0] += 1

        with mts.System(_params(wk, precision, k), w.n_particles.tolist(), w.box) as s:
            en = _run_chunked(s, x, v, n_iter, k, chunk, "aluminium PBC %s" % label, frame)
        p = (2.0 * en[1:, 0, 0] + en[1:, 0, 3] + en[1:, 0, 4]) / (3.0 * vol)
        shell = 4.0 / 3.0 * m.pi * np.diff(np.linspace(0.0, r_max, nbins + 1) ** 3)
        rho = w.n_total / vol
        g = 2.0 * acc / (frames[0] * w.n_total * rho * shell)
        res[label] = {"k": k, "nu": nu, "pressure": p, "rdf": g}
    lo = min(float(r["pressure"].min()) for r in res.values())
    hi = max(float(r["pressure"].max()) for r in res.values())
    edges = np.linspace(lo, hi, 21)
    ref = res["k=1"]["rdf"] if "k=1" in res else None
    out = {}
    centers = 0.5 * (np.linspace(0.0, r_max, nbins + 1)[1:] + np.linspace(0.0, r_max, nbins + 1)[:-1])
    for label, r in res.items():
        g = r["rdf"]
        ipk = int(np.argmax(g))
        out[label] = {"k": r["k"], "nu": r["nu"], "pressure_mean": float(r["pressure"].mean()),
                      "pressure_std": float(r["pressure"].std()), "samples": int(len(r["pressure"])),
                      "pressure_hist": (np.histogram(r["pressure"], bins=edges)[0]
                                        / len(r["pressure"])).tolist(),
                      "rdf_first_peak": [float(centers[ipk]), float(g[ipk])],
                      "rdf_l1_vs_sv": (float(np.abs(g - ref).sum() * (r_max / nbins))
                                       if ref is not None else None),
                      "rdf": g.tolist()}
    return {"experiment": "aluminium parameters, cutoff + PBC: pressure and RDF per step-size "
                          "factor and pure two-body (Sec. 4.2.2, Figs. 6, 7)",
            "n_particles": w.n_total, "box": box.tolist(), "rc_pair": w.rc_pair,
            "rc_triplet": w.rc_triplet, "dt": w.dt, "n_eq": n_eq, "n_iter": n_iter,
            "precision": precision, "pressure_bin_edges": edges.tolist(),
            "rdf_r": centers.tolist(), "runs": out, "data": "synthetic"}


def traffic_probe(w, precision: str, k: int, tune_ms: int):
    """For HBM counter runs (FETCH_SIZE / WRITE_SIZE): four outer cycles of the tuned
    r-RESPA loop with energy records (the triplet launch of the timed region, once per
    cycle), then three copies of a 256 MiB tensor (the calibration kernel: 262,144 KiB
    read and written each)."""
    import torch
    from paper_2507_11172_amd import mts

    dev = torch.device("cuda:0")
    x = torch.tensor(w.x, dtype=torch.float64, device=dev)
    v = torch.tensor(w.v, dtype=torch.float64, device=dev)
    with mts.System(_params(w, precision, k), w.n_particles.tolist(), w.box) as sysm:
        if tune_ms > 0:
            sysm.autotune(x, v, tune_ms)
        e = torch.zeros((5, w.n_systems, mts.MTS_NE), dtype=torch.float64, device=dev)
        sysm.respa_step(x, v, 4 * k, e)
        sysm.sync()
    a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev).fill_(1.0)
    for _ in range(3):
        b = a.clone()
    torch.cuda.synchronize()
    print("traffic probe done (%d-particle workload, calibration copy %d bytes)"
          % (w.n_total, b.numel() * 4), flush=True)


def _counter_rows(path: str):
    """(kernel name, dispatch id, counter value) of a rocprofv3 counter-collection CSV;
    values of one dispatch (one per XCD or instance) are summed."""
    import csv
    acc = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            key = (row["Kernel_Name"], row.get("Dispatch_Id", row.get("Correlation_Id")))
            acc[key] = acc.get(key, 0.0) + float(row["Counter_Value"])
    return acc


def traffic_summary(fetch_csv: str, write_csv: str, kernel: str, workload: str,
                    precision: str, copy_kib: float = 262144.0):
    """HBM bytes per launch of `kernel` (a part of its demangled name) from a FETCH_SIZE and a
    WRITE_SIZE counter run of the traffic probe.  Each counter is scaled by what it reads
    for the probe's plain copy of copy_kib KiB (the largest copy dispatch), so that the
    result is in the same bytes the copy moves; returns the row for profiles/hbm_traffic.json."""
    out = {"workload": workload, "precision": precision, "kernel": kernel,
           "sources_sha": kernel_sources_sha()}
    total = 0.0
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _counter_rows(path)
        copy = max((v for (k, _), v in rows.items() if "copyBuffer" in k), default=0.0)
        vals = [v for (k, _), v in rows.items() if kernel in k]
        if not vals or copy <= 0:
            raise SystemExit("no %s dispatches of %s or of the calibration copy in %s"
                             % (name, kernel, path))
        factor = copy_kib / copy
        per = sum(vals) / len(vals)
        out[name] = {"calibration_copy_kib": copy, "factor": factor, "dispatches": len(vals),
                     "kib_per_dispatch": per, "scaled_kib": per * factor}
        total += per * factor * 1024.0
    out["bytes_per_launch"] = int(round(total))
    return out


def traffic_table(fetch_csv: str, write_csv: str, stats_csv: str = "", copy_kib: float = 262144.0):
    """Markdown table of HBM bytes per dispatch of every kernel in a FETCH_SIZE and a
    WRITE_SIZE counter run, each counter scaled by the plain copy as in traffic_summary;
    with a rocprofv3 kernel-stats CSV, the average duration and the rate they imply."""
    import csv
    per = {}
    for col, path in ((0, fetch_csv), (1, write_csv)):
        rows = _counter_rows(path)
        copy = max((v for (k, _), v in rows.items() if "copyBuffer" in k), default=0.0)
        if copy <= 0:
            raise SystemExit("no calibration copy in %s" % path)
        acc = {}
        for (k, _), v in rows.items():
            acc.setdefault(k, []).append(v * copy_kib / copy)
        for k, vals in acc.items():
            per.setdefault(k, [None, None, 0])
            per[k][col] = sum(vals) / len(vals)
            per[k][2] = max(per[k][2], len(vals))
    avg_us = {}
    if stats_csv:
        with open(stats_csv, newline="") as f:
            for row in csv.DictReader(f):
                avg_us[row["Name"]] = float(row["AverageNs"]) / 1e3
    lines = ["| kernel | dispatches | FETCH MiB | WRITE MiB | total MiB | avg us | GB/s |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for k in sorted(per, key=lambda k: -((per[k][0] or 0) + (per[k][1] or 0))):
        fe, wr, nd = per[k]
        tot = (fe or 0) + (wr or 0)
        us = avg_us.get(k)
        rate = "%.0f" % (tot * 1024 / (us * 1e3)) if us and fe is not None and wr is not None else "-"
        lines.append("| `%s` | %d | %s | %s | %.1f | %s | %s |" % (
            k.split("(")[0].replace("void ", ""), nd,
            "-" if fe is None else "%.1f" % (fe / 1024), "-" if wr is None else "%.1f" % (wr / 1024),
            tot / 1024, "-" if us is None else "%.1f" % us, rate))
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed r-RESPA outer cycles")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="fcc1m")
    ap.add_argument("--precision", default="", choices=["", "fp64", "fp32"],
                    help="default: fp64 for fcc1m, fcc32k and fcc500, the FP32 form otherwise")
    ap.add_argument("--k", type=int, default=0, help="override the step-size factor")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-form", action="store_true")
    ap.add_argument("--tune-ms", type=int, default=3000,
                    help="autotuning budget before the timed region (0: default configuration)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only run the kernels of the HBM counter runs, print no bench line")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="scale the two counter runs of --traffic-probe into HBM bytes per "
                         "launch of --traffic-kernel and print the JSON row")
    ap.add_argument("--traffic-table", nargs="+", metavar="CSV",
                    help="FETCH_CSV WRITE_CSV [KERNEL_STATS_CSV]: print the HBM bytes of every "
                         "kernel of the two counter runs as a markdown table")
    ap.add_argument("--traffic-kernel", default="mts::k_triplet_items<double, false, true, false, true, false, ",
                    help="a part of the demangled name (the register budget, the last template "
                         "argument, is left open)")
    ap.add_argument("--loop-steps", type=int, default=5,
                    help="cycles of the one-handle-per-replica loop (batched workload)")
    ap.add_argument("--rvite-sweep", action="store_true",
                    help="the toy scenario's RVITE study (Sec. 4.2.1) on DirectSum instead of "
                         "the bench line: one JSON line with RVITE per nu and step-size factor")
    ap.add_argument("--sweep-nu", default="0.05,0.1,0.2,0.3,0.5,0.7,1.0")
    ap.add_argument("--sweep-k", default="1,2,3,4,6,8,12")
    ap.add_argument("--sweep-iter", type=int, default=24000,
                    help="inner steps per run (a multiple of every factor)")
    ap.add_argument("--nested-study", action="store_true",
                    help="cost and energy deviation of nested r-RESPA vs plain factors on the "
                         "32,000-particle system instead of the bench line")
    ap.add_argument("--study-iter", type=int, default=10000)
    ap.add_argument("--study-nu", type=float, default=0.073,
                    help="nu of the nested study (<= 0: the workload's own)")
    ap.add_argument("--study-workload", default="fcc32k", choices=["fcc32k", "al4995_pbc"])
    ap.add_argument("--al-energy-study", action="store_true",
                    help="aluminium DirectSum total energy vs Stoermer-Verlet (Fig. 4)")
    ap.add_argument("--al-iter", type=int, default=2400)
    ap.add_argument("--al-pbc-study", action="store_true",
                    help="aluminium cutoff + PBC pressure and RDF per factor (Figs. 6, 7)")
    ap.add_argument("--al-pbc-iter", type=int, default=24000)
    ap.add_argument("--al-pbc-eq", type=int, default=2400)
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this library has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        return 2

    if args.rvite_sweep:
        nus = [float(v) for v in args.sweep_nu.split(",")]
        ks = [int(v) for v in args.sweep_k.split(",")]
        print(json.dumps(rvite_sweep(nus, ks, args.sweep_iter, args.precision or "fp64")),
              flush=True)
        return 0
    if args.al_energy_study:
        print(json.dumps(al_energy_study(args.al_iter, [2, 3, 4, 6, 12],
                                         args.precision or "fp64")), flush=True)
        return 0
    if args.al_pbc_study:
        print(json.dumps(al_pbc_study(args.al_pbc_iter, args.al_pbc_eq, [1, 2, 3, 4, 6, 12],
                                      args.precision or "fp64")), flush=True)
        return 0
    if args.nested_study:
        schemes = [(2, 1, 0.0), (10, 1, 0.0), (2, 5, 2.0), (2, 5, 2.2), (5, 2, 2.0)]
        print(json.dumps(nested_study(args.study_iter, args.study_nu, args.precision or "fp64",
                                      schemes, args.study_workload)), flush=True)
        return 0
    w = _workload(args.workload)
    k = args.k or w.k
    precision = args.precision or w.precision
    if args.traffic_table:
        if len(args.traffic_table) not in (2, 3):
            raise SystemExit("--traffic-table takes FETCH_CSV WRITE_CSV [KERNEL_STATS_CSV]")
        print(traffic_table(*args.traffic_table), flush=True)
        return 0
    if args.traffic_summary:
        kern = args.traffic_kernel.split("<")[0].split("::")[-1]
        row = traffic_summary(args.traffic_summary[0], args.traffic_summary[1],
                              args.traffic_kernel, w.name, precision)
        row["kernel_reported"] = kern
        print(json.dumps(row), flush=True)
        return 0
    if args.traffic_probe:
        traffic_probe(w, precision, k, args.tune_ms)
        return 0
    r = run_gpu(w, precision, k, args.steps, args.warmup, args.tune_ms)
    steps_per_s = w.n_systems * r["inner_steps"] / r["elapsed_s"]
    ms_per_cycle = 1e3 * r["elapsed_s"] / args.steps
    # triplet work and kernel time of one full step (nested: the whole cutoff set once, with
    # its class weights, and the inner class at the other k_outer - 1 cycle ends)
    evaluated = r["triplets_per_eval"] + (w.k_outer - 1) * r["inner_class_triplets"]
    trip_s = r["triplet_ms_per_full_step"] * 1e-3
    achieved = FLOPS_PER_TRIPLET * evaluated / trip_s / 1e12 if trip_s > 0 else 0.0
    peak = PEAK_TFLOPS[precision]
    # list force kernel: algorithmic HBM bytes of one launch over its average duration
    pair_bytes = (PAIR_BYTES_FIXED * w.n_total + PAIR_BYTES_PER_ENTRY * r["list_entries_est"])
    pair_s = r["pair_kernel_ms"] * 1e-3
    kernel = "k_triplet_items"  # one persistent launch per evaluation (with the pair-list
    # build as its last items when tuning["shared_launch"] is 1)
    if w.method == "direct":
        kernel = "k_direct_triplet"
    if w.k_outer > 1:
        kernel += " + inner-class passes"
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
        "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "method": w.method, "n_particles": w.n_total,
                   "n_systems": w.n_systems,
                   "k": k, "inner_steps": r["inner_steps"], "precision": precision,
                   "rc_pair": w.rc_pair, "rc_triplet": w.rc_triplet, "nu": w.nu, "dt": w.dt,
                   "step": "one r-RESPA outer cycle (k inner steps + 1 triplet evaluation)"},
        "triplets_per_s": evaluated / trip_s if trip_s > 0 else None,
        "triplets_per_eval": r["triplets_per_eval"],
        "kernel_ms": {"triplet": r["triplet_kernel_ms"], "pair": r["pair_kernel_ms"]},
        "energy_drift_per_particle": r["energy_drift_per_particle"],
        "rvite": r["rvite"],
        "roofline": {"bound": "alu", "kernel": kernel, "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": stored_traffic(w.name, precision, kernel),
                     "flops_per_triplet": FLOPS_PER_TRIPLET,
                     "triplets_per_launch": evaluated / max(r["triplet_launches_per_full_step"], 1),
                     "launch_ms": r["triplet_kernel_ms"]},
        "pair_roofline": {"bound": "hbm", "kernel": "k_pair_list",
                          "achieved": pair_bytes / pair_s / 1e9 if pair_s > 0 else None,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": pair_bytes / pair_s / 1e9 / HBM_PEAK_GBS if pair_s > 0 else None,
                          "algorithmic_bytes_per_launch": pair_bytes,
                          "bytes": "%d B per particle + %d B per list entry (list length "
                                   "estimated as rho 4/3 pi (rc + skin)^3)"
                                   % (PAIR_BYTES_FIXED, PAIR_BYTES_PER_ENTRY),
                          "launch_ms": r["pair_kernel_ms"]},
        "tuning": r["tuning"],
    }
    if w.k_outer > 1:
        out["config"].update({
            "k_outer": w.k_outer, "rc_triplet_inner": w.rc_triplet_inner,
            "step": "one full step of nested r-RESPA: k_outer cycles of k inner steps; the "
                    "inner triplet class (all edges <= rc_triplet_inner) every k steps, the "
                    "whole cutoff set every k * k_outer"})
        out["inner_class_triplets"] = r["inner_class_triplets"]
    if w.n_systems > 1:
        out["per_system_loop"] = {
            "value": run_per_system_loop(w, precision, k, args.loop_steps),
            "unit": "MD steps/s", "cycles": args.loop_steps,
            "note": "the same replicas, one handle each, stepped one after another"}
    if not args.no_fp32_form and precision == "fp64":
        r32 = run_gpu(w, "fp32", k, args.steps, args.warmup, args.tune_ms)
        t32 = r32["triplet_ms_per_full_step"] * 1e-3
        ev32 = r32["triplets_per_eval"] + (w.k_outer - 1) * r32["inner_class_triplets"]
        out["fp32_form"] = {
            "value": w.n_systems * r32["inner_steps"] / r32["elapsed_s"], "unit": "MD steps/s",
            "triplets_per_s": ev32 / t32 if t32 > 0 else None,
            "kernel_ms": {"triplet": r32["triplet_kernel_ms"], "pair": r32["pair_kernel_ms"]},
            "roofline_frac_fp32_peak": (FLOPS_PER_TRIPLET * ev32 / t32 / 1e12
                                        / PEAK_TFLOPS["fp32"]) if t32 > 0 else None,
            # this library emits no packed FP32: its FP32 arithmetic issues at the FP64
            # vector rate, the reachable ceiling
            "roofline_frac_unpacked_fp32": (FLOPS_PER_TRIPLET * ev32 / t32 / 1e12
                                            / PEAK_TFLOPS["fp64"]) if t32 > 0 else None,
            "speedup_vs_fp64": (w.n_systems * r32["inner_steps"] / r32["elapsed_s"]) / steps_per_s,
            "energy_drift_per_particle": r32["energy_drift_per_particle"],
            "rvite": r32["rvite"],
            "error_vs_fp64": fp32_force_error(w, k),
        }
    if precision == "fp32":  # an FP32-form line states its error against the FP64 path
        out["error_vs_fp64"] = fp32_force_error(w, k)
    if not args.no_cpu_baseline:
        if w.n_systems == 1 and w.n_total <= 40_000:
            out["cpu_baseline"] = cpu_baseline(w, k)
        elif w.n_systems == 1 and w.method != "direct" and w.k_outer == 1:
            out["cpu_baseline"] = cpu_baseline_subset(w, k)
        else:
            out["cpu_baseline"] = None  # the brute-force oracle is O(N^2) or worse here
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
