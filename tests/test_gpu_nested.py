"""GPU parity of nested r-RESPA (three time scales over two triplet distance classes) and
of Algorithm 1's sub-step form against the FP64 CPU oracle.

The HIP path evaluates the inner class (all edges <= r_a) every k steps and, at full steps
(every k * k_outer), the whole cutoff set as well; it gathers F_in + k_outer (F - F_in),
while the oracle sums each class on its own and applies the two kicks one after the other.
The two agree to round-off amplified over the run: the bars of the two-level trajectory
tests (positions within 1e-10, velocities and energy records within 1e-10 relative).
"""
import numpy as np
import pytest

import oracle
from paper_2507_11172_amd import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    return torch


def _dev(a):
    torch = _torch()
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _params(w, **kw):
    from paper_2507_11172_amd import mts
    return mts.Params(epsilon=w.epsilon, sigma=w.sigma, rc_pair=w.rc_pair, nu=w.nu,
                      rc_triplet=w.rc_triplet, mass=w.mass, dt=kw.pop("dt", w.dt), **kw)


def _small_box(n=150, length=6.2, seed=3):
    rng = W.rng_for(seed)
    x, box = W.fcc_subset(n, n / length ** 3, 0.05, rng)
    v = W.maxwell_boltzmann(n, 0.7, rng)
    return W.Workload("smallbox", x, v, box[None, :], np.array([n]), np.array([0.7]))


CASES = {"fcc500": W.plain_fp64, "smallbox": _small_box,
         "fcc256": lambda: W.fcc_workload("fcc256", 4, 17, jitter=0.15)}


def _run(w, n_iter, graph=True, **kw):
    torch = _torch()
    from paper_2507_11172_amd import mts
    p = _params(w, **kw)
    with mts.System(p, w.n_particles.tolist(), w.box) as s:
        s.set_option(mts.MTS_OPT_CYCLE_GRAPH, int(graph))
        x, v = _dev(w.x), _dev(w.v)
        e = torch.zeros((n_iter // p.span + 1, w.n_systems, mts.MTS_NE), dtype=torch.float64,
                        device="cuda")
        s.respa_step(x, v, n_iter, e)
        s.sync()
        return x.cpu().numpy(), v.cpu().numpy(), e.cpu().numpy()


def _assert_trajectory(got, ref, box):
    (x, v, e), (xo, vo, eo) = got, ref
    dx = x - xo
    dx -= box * np.rint(dx / box)
    assert np.abs(dx).max() <= 1e-10
    assert np.abs(v - vo).max() <= 1e-10 * np.abs(vo).max()
    assert np.abs(e - eo).max() <= 1e-10 * np.abs(eo).max()


@pytest.mark.parametrize("case,skin,k,k_outer,r_a,n_iter", [
    ("fcc500", 0.0, 2, 3, 2.0, 24),    # pair list (default skin), r_a inside the first shells
    ("fcc256", 0.6, 3, 2, 2.2, 18),    # wide skin, odd k (F2 buffers alternate per cycle)
    ("smallbox", 0.01, 2, 2, 1.8, 16),  # no pair list, two cells per edge
    ("fcc500", 0.0, 1, 4, 1.5, 16),    # k = 1: the inner class every step
])
def test_nested_respa_matches_oracle(case, skin, k, k_outer, r_a, n_iter):
    w = CASES[case]()
    box = w.box[0]
    ref = oracle.respa_nested(w.x, w.v, box, n_iter=n_iter, k=k, k_outer=k_outer, r_a=r_a)
    got = _run(w, n_iter, k=k, k_outer=k_outer, rc_triplet_inner=r_a, skin=skin)
    assert got[2].shape == (n_iter // (k * k_outer) + 1, 1, 5)
    _assert_trajectory((got[0], got[1], got[2][:, 0, :]), ref, box)


def test_nested_graph_matches_eager_bitwise():
    """Graphs of mid and full cycles replayed over two calls equal eager launches."""
    w = W.plain_fp64()
    kw = dict(k=3, k_outer=2, rc_triplet_inner=2.0)
    a = _run(w, 24, graph=True, **kw)
    b = _run(w, 24, graph=False, **kw)
    for p, q in zip(a, b):
        assert np.array_equal(p, q)


def test_nested_fp32_form():
    """FP32 arithmetic in both classes: the trajectory stays within FP32 force error of
    the oracle's over a short run."""
    w = W.plain_fp64()
    box = w.box[0]
    xo, vo, eo = oracle.respa_nested(w.x, w.v, box, n_iter=12, k=2, k_outer=3, r_a=2.0)
    x, v, e = _run(w, 12, k=2, k_outer=3, rc_triplet_inner=2.0, precision="fp32")
    dx = x - xo
    dx -= box * np.rint(dx / box)
    assert np.abs(dx).max() <= 1e-7
    assert np.abs(v - vo).max() <= 1e-5 * np.abs(vo).max()
    tot, toto = e[:, 0, :3].sum(axis=1), eo[:, :3].sum(axis=1)
    assert np.abs(tot - toto).max() / w.n_total <= 1e-6


def test_nested_batched_matches_single_systems():
    """A batch of uneven replicas under nested r-RESPA equals each replica on its own, bit
    for bit."""
    w = W.batched(n_replicas=3, n_min=300, n_max=1500)
    kw = dict(k=2, k_outer=2, rc_triplet_inner=2.0, skin=0.3)
    xb, vb, eb = _run(w, 8, **kw)
    off = 0
    for r in range(w.n_systems):
        n = int(w.n_particles[r])
        sl = slice(off, off + n)
        wr = W.Workload("rep%d" % r, w.x[sl], w.v[sl], w.box[r:r + 1], np.array([n]),
                        w.temperature[r:r + 1])
        x, v, e = _run(wr, 8, **kw)
        assert np.array_equal(xb[sl], x) and np.array_equal(vb[sl], v), r
        assert np.array_equal(eb[:, r, :], e[:, 0, :]), r
        off += n


def test_algorithm1_substeps_on_respa_step():
    """Algorithm 1 with full step delta_t and P sub-steps is respa_step with dt = delta_t / P
    and k = P: the GPU run follows the oracle's Algorithm 1 as printed."""
    w = W.plain_fp64()
    box = w.box[0]
    P, n_outer, delta_t = 4, 5, 0.004
    ref = oracle.respa_alg1(w.x, w.v, box, n_outer=n_outer, P=P, delta_t=delta_t)
    x, v, e = _run(w, n_outer * P, k=P, dt=delta_t / P)
    _assert_trajectory((x, v, e[:, 0, :]), ref, box)


def test_nested_step_count_must_span_full_steps():
    torch = _torch()
    from paper_2507_11172_amd import mts
    w = W.plain_fp64()
    p = _params(w, k=2, k_outer=3, rc_triplet_inner=2.0)
    with mts.System(p, w.n_particles.tolist(), w.box) as s:
        x, v = _dev(w.x), _dev(w.v)
        with pytest.raises(mts.MTSError) as e:
            s.respa_step(x, v, 4)
        assert e.value.code == mts.MTS_ERR_NOT_MULTIPLE_OF_K
        s.respa_step(x, v, 6)
        s.sync()
        assert bool(torch.isfinite(x).all())


def test_nested_study_short():
    """The nested study's runner on a short horizon: Stoermer-Verlet deviates from itself by
    zero, every scheme's records are finite."""
    import math
    import bench
    r = bench.nested_study(100, 0.073, "fp64", [(2, 1, 0.0), (2, 5, 2.0)])
    s = r["schemes"]
    assert [(q["k"], q["k_outer"]) for q in s] == [(1, 1), (2, 1), (2, 5)]
    assert s[0]["mean_rel_dev_vs_sv"] == 0.0
    for q in s:
        assert math.isfinite(q["mean_rel_dev_vs_sv"]) and q["steps_per_s"] > 0


def _class_batch():
    """Systems whose triplet tiles fall into different tile classes (liquid density with
    five cells per edge, a small dense box with two large cells per edge, one between)."""
    specs = [(2048, 0.8, 71), (365, 0.9, 72), (1200, 0.7, 73)]
    xs, vs, boxes = [], [], []
    for n, rho, seed in specs:
        rng = W.rng_for(seed)
        x, box = W.fcc_subset(n, rho, 0.05, rng)
        xs.append(x)
        vs.append(W.maxwell_boltzmann(n, 0.8, rng))
        boxes.append(box)
    return W.Workload("classes", np.concatenate(xs), np.concatenate(vs), np.stack(boxes),
                      np.array([n for n, _, _ in specs]), np.full(len(specs), 0.8))


def test_nested_tile_classes_after_autotune():
    """Nested r-RESPA on a batch of very different tiles (one system staged whole), after
    the autotuner has picked its configuration: every system follows the oracle's nested
    trajectory."""
    torch = _torch()
    from paper_2507_11172_amd import mts
    w = _class_batch()
    k, k_outer, r_a, n_iter = 2, 2, 2.0, 8
    p = _params(w, k=k, k_outer=k_outer, rc_triplet_inner=r_a, skin=0.3)
    with mts.System(p, w.n_particles.tolist(), w.box) as s:
        assert s.tuning()["tile_classes"] == 1
        x, v = _dev(w.x), _dev(w.v)
        s.autotune(x, v, 300)
        e = torch.zeros((n_iter // (k * k_outer) + 1, w.n_systems, mts.MTS_NE),
                        dtype=torch.float64, device="cuda")
        s.respa_step(x, v, n_iter, e)
        s.sync()
        xb, vb, eb = x.cpu().numpy(), v.cpu().numpy(), e.cpu().numpy()
    off = 0
    for r in range(w.n_systems):
        n = int(w.n_particles[r])
        sl = slice(off, off + n)
        ref = oracle.respa_nested(w.x[sl], w.v[sl], w.box[r], n_iter=n_iter, k=k,
                                  k_outer=k_outer, r_a=r_a)
        _assert_trajectory((xb[sl], vb[sl], eb[:, r, :]), ref, w.box[r])
        off += n


def test_nested_without_inner_triplets_is_algorithm2_at_32k():
    """32,000 particles in the bench's nested launch configuration, with the split below
    every distance (empty inner class): the run equals Algorithm 2 with s = k * k_outer up
    to summation order (pair lists are rebuilt on different schedules)."""
    w = W.nested_at_scale()
    box = w.box[0]
    a = _run(w, 20, k=2, k_outer=5, rc_triplet_inner=0.5)
    b = _run(w, 20, k=10)
    d = a[0] - b[0]
    d -= box * np.rint(d / box)
    assert np.abs(d).max() <= 1e-10
    assert np.abs(a[1] - b[1]).max() <= 1e-10 * np.abs(b[1]).max()
    assert np.abs(a[2] - b[2]).max() <= 1e-10 * np.abs(b[2]).max()


@pytest.mark.slow
def test_nested_at_scale_32k_vs_oracle():
    """32,000 particles, split at 2.0, k = 2, k_outer = 2: one full step against the
    oracle's nested loop on the whole system (five class evaluations of 32,000 particles
    on the host, about a minute)."""
    w = W.nested_at_scale()
    box = w.box[0]
    print("oracle nested run, 32,000 particles", flush=True)
    ref = oracle.respa_nested(w.x, w.v, box, n_iter=4, k=2, k_outer=2, r_a=2.0)
    got = _run(w, 4, k=2, k_outer=2, rc_triplet_inner=2.0)
    _assert_trajectory((got[0], got[1], got[2][:, 0, :]), ref, box)


def _triangle(order, eps):
    tri = np.array([[10.0, 10.0, 10.0], [11.5 + eps, 10.0, 10.0], [10.75, 10.75, 10.0]])
    x = tri[list(order)]
    return W.Workload("triangle", x, np.zeros_like(x), np.full((1, 3), 40.0), np.array([3]),
                      np.array([0.0]))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("order", [(0, 1, 2), (2, 0, 1)])
@pytest.mark.parametrize("offset", [0.0, 1.0])
def test_nested_class_split_is_exact(precision, order, offset):
    """One triangle whose longest edge lies exactly at the split r_a = 1.5 (squared 2.25,
    exact in binary: inner class) or just beyond it, inside the band where the kernel
    settles the class with the canonical FP64 displacement (outer class).  The input order
    makes that edge an anchor edge (0, 1, 2) or the j-k edge (2, 0, 1).  The edge grows past
    1.5 during the first step, so the class taken at x^0 decides whether the triplet's
    first kick pairs with later ones: the other class changes the velocities at first
    order (checked on the oracle), far beyond the bar."""
    eps = (2.0 ** -42 if precision == "fp64" else 2.0 ** -20) * offset
    w = _triangle(order, eps)
    box = w.box[0]
    assert oracle.triplet_forces(w.x, box, rc=1.5).count == (1 if offset == 0.0 else 0)
    ref = oracle.respa_nested(w.x, w.v, box, n_iter=3, k=1, k_outer=3, r_a=1.5)
    if offset == 0.0:   # outer at x^0, as later: a split just below the edge
        other = oracle.respa_nested(w.x, w.v, box, n_iter=3, k=1, k_outer=3, r_a=1.4999)
    else:               # inner at x^0, outer later: the triangle without the offset
        w0 = _triangle(order, 0.0)
        other = oracle.respa_nested(w0.x, w0.v, box, n_iter=3, k=1, k_outer=3, r_a=1.5)
    tol = 1e-10 if precision == "fp64" else 1e-4
    scale = np.abs(ref[1]).max()
    assert np.abs(other[1] - ref[1]).max() > 10 * tol * scale
    xg, vg, eg = _run(w, 3, k=1, k_outer=3, rc_triplet_inner=1.5, precision=precision)
    assert np.abs(vg - ref[1]).max() <= tol * scale
