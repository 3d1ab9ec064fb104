"""Pins the oracle's r-RESPA loop (Sec. 4.1, Algorithm 2) against textbook velocity
Verlet and against special cases where r-RESPA reduces to it exactly."""
import numpy as np
import pytest

from paper_2507_11172_amd import workloads as W


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_respa_k1_is_velocity_verlet(orc):
    """With s = 1 the two half kicks of F3 merge with the F2 update into one velocity
    Verlet step of the total force: equal up to rounding over 100 steps of 500 particles."""
    w = W.plain_fp64()
    x1, v1, e1 = orc.respa(w.x, w.v, w.box[0], n_iter=100, k=1)
    x2, v2, e2 = orc.velocity_verlet(w.x, w.v, w.box[0], n_iter=100)
    assert _rel(x1, x2) <= 1e-12
    assert _rel(v1, v2) <= 1e-12
    assert np.abs(e1 - e2).max() <= 1e-10 * np.abs(e2).max()


def test_respa_without_three_body_is_velocity_verlet(orc):
    """nu = 0: F3 vanishes and any step-size factor gives plain velocity Verlet on F2."""
    w = W.plain_fp64()
    x1, v1, _ = orc.respa(w.x, w.v, w.box[0], n_iter=40, k=5, nu=0.0)
    x2, v2, _ = orc.velocity_verlet(w.x, w.v, w.box[0], n_iter=40, nu=0.0)
    assert _rel(x1, x2) <= 1e-12
    assert _rel(v1, v2) <= 1e-12


@pytest.mark.parametrize("k", [2, 4])
def test_respa_without_pair_force_is_verlet_with_outer_step(orc, k):
    """eps = 0: only F3 acts, the k inner steps are pure drifts, and Algorithm 2 is velocity
    Verlet with time step k*dt on F3 -- this pins the dt*s/(2m) kick and where it lands."""
    w = W.plain_fp64()
    kw = dict(eps=0.0, nu=0.5)
    x1, v1, e1 = orc.respa(w.x, w.v, w.box[0], n_iter=6 * k, k=k, **kw)
    x2, v2, e2 = orc.velocity_verlet(w.x, w.v, w.box[0], n_iter=6, dt=k * 0.001, **kw)
    assert _rel(x1, x2) <= 1e-11
    assert _rel(v1, v2) <= 1e-11
    assert np.abs(e1[:, 2] - e2[:, 2]).max() <= 1e-11 * np.abs(e2[:, 2]).max()


def test_energy_rows_and_initial_record(orc):
    w = W.plain_fp64()
    _, _, e = orc.respa(w.x, w.v, w.box[0], n_iter=20, k=5)
    assert e.shape == (5, 5)
    p = orc.pair_forces(w.x, w.box[0])
    t = orc.triplet_forces(w.x, w.box[0])
    assert e[0, 0] == pytest.approx(0.5 * np.sum(w.v ** 2), rel=1e-14)
    assert e[0, 1] == pytest.approx(p.energy, rel=1e-14)
    assert e[0, 2] == pytest.approx(t.energy, rel=1e-14)
    assert e[0, 3] == pytest.approx(p.virial, rel=1e-14)
    assert e[0, 4] == pytest.approx(9.0 * t.energy, rel=1e-12)  # Euler: W3 = 9 U3
    assert np.all(e[:, 0] > 0)


def test_checkpoint_resume_is_bitwise(orc):
    """Algorithm 2 recomputes both forces at entry, so two half runs equal one full run."""
    w = W.plain_fp64()
    xa, va, ea = orc.respa(w.x, w.v, w.box[0], n_iter=20, k=5)
    xb, vb, eb = orc.respa(w.x, w.v, w.box[0], n_iter=10, k=5)
    xb, vb, eb2 = orc.respa(xb, vb, w.box[0], n_iter=10, k=5)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    assert np.array_equal(ea[2:], eb2)  # row 0 of the second half is the state at step 10


def test_time_reversibility(orc):
    w = W.plain_fp64()
    x1, v1, _ = orc.respa(w.x, w.v, w.box[0], n_iter=30, k=5)
    x2, v2, _ = orc.respa(x1, -v1, w.box[0], n_iter=30, k=5)
    d = x2 - w.x
    d -= w.box[0] * np.rint(d / w.box[0])
    assert np.abs(d).max() <= 1e-9
    assert _rel(-v2, w.v) <= 1e-9


def _cluster():
    """19-particle FCC cluster (a site and its two nearest shells) in a large box with a
    cutoff beyond the cluster size, so no pair or triplet crosses the cutoff."""
    x, _ = W.fcc(4, 0.8, 0.0, None)
    c = x[np.argmin(np.sum((x - x.mean(axis=0)) ** 2, axis=1))]
    sel = x[np.sum((x - c) ** 2, axis=1) <= 1.8 ** 2]
    box = np.full(3, 40.0)
    return sel - c + 20.0, box


@pytest.mark.parametrize("k", [1, 3])
def test_energy_error_is_second_order(orc, k):
    x, box = _cluster()
    assert x.shape[0] == 19
    v = W.maxwell_boltzmann(19, 0.3, W.rng_for(77))
    kw = dict(rc_pair=9.0, rc3=9.0, nu=0.5, shift=False)
    errs = []
    for dt in (0.004, 0.002):
        n = int(round(0.48 / dt))
        n -= n % k
        _, _, e = orc.respa(x, v, box, n_iter=n, k=k, dt=dt, **kw)
        tot = e[:, 0] + e[:, 1] + e[:, 2]
        errs.append(np.abs(tot - tot[0]).max())
    assert 3.0 <= errs[0] / errs[1] <= 5.0


def test_bounded_nve_energy_fluctuation(orc):
    w = W.plain_fp64()
    _, _, e = orc.respa(w.x, w.v, w.box[0], n_iter=100, k=5)
    tot = e[:, 0] + e[:, 1] + e[:, 2]
    assert np.abs(tot - tot[0]).max() <= 1e-3 * np.mean(e[:, 0])


def test_rvite_definition(orc):
    # Eq. 4: (1 / (K J)) sum |e(i) - mean(e)|
    assert orc.rvite([1.0, 2.0, 3.0], [2.0, 2.0, 2.0]) == pytest.approx(1.0 / 3.0)
    assert orc.rvite([5.0, 5.0], [1.0, 3.0]) == 0.0
