"""Pins the oracle's nested r-RESPA pieces: the triplet distance classes (the intermediate
cutoffs of Sec. 5, after the related work of Sec. 3), the three-level nested loop over
them (Sec. 2.3.1 extended by one level) and Algorithm 1 with P sub-steps.

Each pin reduces to something fixed independently: a hand-placed triangle, the partition
of T(rc) into two disjoint classes, the two-level loop of Algorithm 2 (itself pinned
against velocity Verlet), time reversibility and second-order energy error."""
import numpy as np
import pytest

from paper_2507_11172_amd import workloads as W


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _triangle(pts):
    box = np.full(3, 20.0)
    return np.asarray(pts, dtype=np.float64) + 5.0, box


def test_single_triplet_class_by_longest_edge(orc):
    """Edges 1.2, 1.3 and sqrt(1.2^2 + 1.3^2) = 1.769: inner for a split above 1.769, outer
    below it; the outer class of a split at 1.5 holds the whole triplet."""
    x, box = _triangle([[0, 0, 0], [1.2, 0, 0], [0, 1.3, 0]])
    full = orc.triplet_forces(x, box, rc=2.5)
    assert full.count == 1
    outer = orc.triplet_forces(x, box, rc=2.5, r_lo=1.5)
    assert outer.count == 1 and np.array_equal(outer.f, full.f) and outer.energy == full.energy
    assert orc.triplet_forces(x, box, rc=2.5, r_lo=1.8).count == 0
    assert np.all(orc.triplet_forces(x, box, rc=2.5, r_lo=1.8).f == 0.0)
    assert orc.triplet_forces(x, box, rc=1.5).count == 0     # inner class of a 1.5 split
    assert orc.triplet_forces(x, box, rc=1.8).count == 1     # inner class of a 1.8 split


def test_class_boundary_is_inclusive_on_the_inner_side(orc):
    """Longest edge exactly 1.5 (squared 2.25, exact in binary): inner class of a split at
    1.5, not outer."""
    x, box = _triangle([[0, 0, 0], [1.5, 0, 0], [0.75, 0.5, 0]])
    assert orc.triplet_forces(x, box, rc=1.5).count == 1
    assert orc.triplet_forces(x, box, rc=2.5, r_lo=1.5).count == 0


@pytest.mark.parametrize("r_a", [1.2, 2.0, 2.4])
def test_classes_partition_the_cutoff_set(orc, r_a):
    """Inner (longest edge <= r_a) and outer (r_a < longest edge <= rc) classes are disjoint
    and cover T(rc): counts add exactly; forces, energies and virials add up to rounding."""
    w = W.plain_fp64()
    box = w.box[0]
    full = orc.triplet_forces(w.x, box, rc=2.5)
    inner = orc.triplet_forces(w.x, box, rc=r_a)
    outer = orc.triplet_forces(w.x, box, rc=2.5, r_lo=r_a)
    assert inner.count > 0 and outer.count > 0
    assert inner.count + outer.count == full.count
    assert _rel(inner.f + outer.f, full.f) <= 1e-13
    assert abs(inner.energy + outer.energy - full.energy) <= 1e-13 * abs(full.energy)
    assert abs(inner.virial + outer.virial - full.virial) <= 1e-13 * abs(full.virial)


def test_nested_with_one_outer_step_is_algorithm2(orc):
    """k_outer = 1: both class kicks share the coefficient dt k / 2m, so their sum is the
    F3 kick of Algorithm 2."""
    w = W.plain_fp64()
    x1, v1, e1 = orc.respa_nested(w.x, w.v, w.box[0], n_iter=12, k=3, k_outer=1, r_a=2.0)
    x2, v2, e2 = orc.respa(w.x, w.v, w.box[0], n_iter=12, k=3)
    assert e1.shape == e2.shape == (5, 5)
    assert _rel(x1, x2) <= 1e-12 and _rel(v1, v2) <= 1e-12
    assert np.abs(e1 - e2).max() <= 1e-10 * np.abs(e2).max()


def test_nested_with_empty_inner_class_is_algorithm2_over_the_outer_step(orc):
    """r_a below every distance: only the outer class acts, every k * k_outer steps --
    Algorithm 2 with s = k * k_outer."""
    w = W.plain_fp64()
    for r_a in (0.0, 0.5):
        x1, v1, e1 = orc.respa_nested(w.x, w.v, w.box[0], n_iter=12, k=2, k_outer=3, r_a=r_a)
        x2, v2, e2 = orc.respa(w.x, w.v, w.box[0], n_iter=12, k=6)
        assert _rel(x1, x2) <= 1e-12 and _rel(v1, v2) <= 1e-12
        assert np.abs(e1 - e2).max() <= 1e-10 * np.abs(e2).max()


def test_nested_with_empty_outer_class_is_algorithm2_over_the_inner_step(orc):
    """r_a >= rc3: the outer class is empty, the inner one is all of T(rc3) every k steps;
    energy rows are kept every k * k_outer steps."""
    w = W.plain_fp64()
    x1, v1, e1 = orc.respa_nested(w.x, w.v, w.box[0], n_iter=12, k=2, k_outer=3, r_a=2.5)
    x2, v2, e2 = orc.respa(w.x, w.v, w.box[0], n_iter=12, k=2)
    assert _rel(x1, x2) <= 1e-12 and _rel(v1, v2) <= 1e-12
    assert np.abs(e1 - e2[::3]).max() <= 1e-10 * np.abs(e2).max()


def test_nested_is_time_reversible(orc):
    """The nested impulse method is symmetric: running back with -v retraces the path (a
    misplaced or unpaired half kick breaks this)."""
    w = W.plain_fp64()
    box = w.box[0]
    x1, v1, _ = orc.respa_nested(w.x, w.v, box, n_iter=24, k=2, k_outer=3, r_a=2.0)
    assert _rel(x1, w.x) > 1e-6
    x2, v2, _ = orc.respa_nested(x1, -v1, box, n_iter=24, k=2, k_outer=3, r_a=2.0)
    d = x2 - w.x
    d -= box * np.rint(d / box)
    assert np.abs(d).max() <= 1e-9
    assert _rel(-v2, w.v) <= 1e-9


def _trimer_and_one():
    """An LJ trimer (equilateral, edge 1.12) and a fourth particle 2.0 from each of its
    atoms, in a large box with cutoffs beyond the cluster: the trimer's own triplet is in
    the inner class of a split at 1.5, the three triplets holding the fourth particle in
    the outer class, and over a short cold run no edge comes near 1.5."""
    r = 1.12 / np.sqrt(3.0)
    tri = [[r * np.cos(t), r * np.sin(t), 0.0] for t in (0.0, 2 * np.pi / 3, 4 * np.pi / 3)]
    x = np.vstack([tri, [[0.0, 0.0, np.sqrt(4.0 - r * r)]]]) + 20.0
    return x, np.full(3, 40.0)


def _edges(x):
    d = np.sqrt(np.sum((x[:, None] - x[None]) ** 2, axis=-1))
    return d[0, 1], d[0, 2], d[1, 2], min(d[0, 3], d[1, 3], d[2, 3])


def test_nested_energy_error_is_second_order(orc):
    x, box = _trimer_and_one()
    v = W.maxwell_boltzmann(4, 0.05, W.rng_for(77))
    kw = dict(rc_pair=9.0, rc3=9.0, nu=0.5, shift=False)
    xs, vs = x, v
    for _ in range(60):  # the class of every triplet stays put along the coarser run
        xs, vs, _ = orc.respa_nested(xs, vs, box, n_iter=4, k=2, k_outer=2, r_a=1.5, dt=0.002,
                                     **kw)
        e = _edges(xs)
        assert max(e[:3]) < 1.3 and e[3] > 1.7
    errs = []
    for dt in (0.004, 0.002):
        n = int(round(0.48 / dt))
        _, _, e = orc.respa_nested(x, v, box, n_iter=n, k=2, k_outer=2, r_a=1.5, dt=dt, **kw)
        tot = e[:, 0] + e[:, 1] + e[:, 2]
        errs.append(np.abs(tot - tot[0]).max())
    assert 3.0 <= errs[0] / errs[1] <= 5.0


def test_algorithm1_with_substeps_is_algorithm2(orc):
    """Algorithm 1 with full step delta_t and P sub-steps performs the same operations as
    Algorithm 2 with dt = delta_t / P and s = P (the paper's single-loop simplification)."""
    w = W.plain_fp64()
    box = w.box[0]
    x1, v1, e1 = orc.respa_alg1(w.x, w.v, box, n_outer=5, P=4, delta_t=0.004)
    x2, v2, e2 = orc.respa(w.x, w.v, box, n_iter=20, k=4, dt=0.001)
    assert e1.shape == e2.shape == (6, 5)
    assert _rel(x1, x2) <= 1e-12 and _rel(v1, v2) <= 1e-12
    assert np.abs(e1 - e2).max() <= 1e-10 * np.abs(e2).max()


def test_algorithm1_with_one_substep_is_velocity_verlet(orc):
    w = W.plain_fp64()
    x1, v1, _ = orc.respa_alg1(w.x, w.v, w.box[0], n_outer=10, P=1, delta_t=0.001)
    x2, v2, _ = orc.velocity_verlet(w.x, w.v, w.box[0], n_iter=10, dt=0.001)
    assert _rel(x1, x2) <= 1e-12 and _rel(v1, v2) <= 1e-12


def test_nested_argument_checks(orc):
    w = W.plain_fp64()
    with pytest.raises(orc.OracleError) as e:
        orc.respa_nested(w.x, w.v, w.box[0], n_iter=10, k=2, k_outer=3, r_a=2.0)
    assert e.value.code == orc.ERR_NOT_MULTIPLE_OF_K
    with pytest.raises(orc.OracleError) as e:
        orc.respa_nested(w.x, w.v, w.box[0], n_iter=12, k=2, k_outer=0, r_a=2.0)
    assert e.value.code == orc.ERR_INVALID_ARG
