"""Pins the oracle's many-particle force sums: cutoff sets, periodic images, N3 and energies."""
import itertools
import math

import numpy as np
import pytest

from paper_2507_11172_amd import workloads as W


def _jittered(n_cells=4, density=0.8, jitter=0.1, seed=5):
    x, box = W.fcc(n_cells, density, jitter, W.rng_for(seed))
    return x, box


def _min_edge_gap(x, box, p, rc):
    d = x - x[p]
    d -= box * np.rint(d / box)
    r = np.sqrt(np.sum(d * d, axis=1))
    r[p] = np.inf
    return np.min(np.abs(r - rc))


@pytest.mark.parametrize("kind", ["pair", "triplet"])
def test_forces_are_minus_gradient_of_energy(orc, kind):
    """Central differences on the total energy, relative error below 1e-6."""
    x, box = _jittered()
    rc, h = 2.5, 1e-5
    if kind == "pair":
        total = lambda y: orc.pair_forces(y, box, rc=rc, shift=False)
    else:
        total = lambda y: orc.triplet_forces(y, box, rc=rc)
    f = total(x).f
    scale = np.sqrt(np.mean(np.sum(f * f, axis=1)))
    rng = np.random.default_rng(1)
    checked = 0
    for p in rng.choice(x.shape[0], size=40, replace=False):
        if _min_edge_gap(x, box, p, rc) < 4 * h:
            continue  # the truncated energy jumps at the cutoff
        for c in range(3):
            xp = x.copy(); xp[p, c] += h
            xm = x.copy(); xm[p, c] -= h
            num = -(total(xp).energy - total(xm).energy) / (2 * h)
            assert abs(num - f[p, c]) <= 1e-6 * max(scale, abs(f[p, c]))
        checked += 1
        if checked == 8:
            break
    assert checked >= 4


def test_newton_third_law_and_invariances(orc):
    x, box = _jittered(seed=9)
    for fn in (lambda y: orc.pair_forces(y, box), lambda y: orc.triplet_forces(y, box)):
        r = fn(x)
        mag = np.sum(np.abs(r.f))
        assert np.abs(r.f.sum(axis=0)).max() <= 1e-12 * mag
        # translation (positions re-wrapped into the box)
        t = fn(np.mod(x + np.array([0.37, -1.91, 2.53]), box))
        assert np.abs(t.f - r.f).max() <= 1e-11 * np.abs(r.f).max()
        assert t.count == r.count
        assert t.energy == pytest.approx(r.energy, rel=1e-12)
        # permutation of labels permutes the forces
        perm = np.random.default_rng(2).permutation(x.shape[0])
        q = fn(x[perm])
        assert np.abs(q.f - r.f[perm]).max() <= 1e-11 * np.abs(r.f).max()
        assert q.count == r.count
        assert q.energy == pytest.approx(r.energy, rel=1e-12)


def _fcc_shell(density, rc):
    """Lattice vectors of an infinite FCC crystal within rc of the origin (origin excluded)."""
    a = (4.0 / density) ** (1.0 / 3.0)
    m = int(math.ceil(rc / a)) + 1
    pts = []
    for i, j, k in itertools.product(range(-m, m + 1), repeat=3):
        for b in W.FCC_BASIS:
            p = (np.array([i, j, k], dtype=float) + b) * a
            r = np.linalg.norm(p)
            if 0.0 < r <= rc:
                pts.append(p)
    return np.array(pts)


def _atm_poly(p0, p1, p2, nu):
    """phi3 = nu [P^-3/2 + 3/8 T P^-5/2] from squared edges (law-of-cosines route)."""
    a = np.sum((p1 - p0) ** 2)
    b = np.sum((p2 - p0) ** 2)
    c = np.sum((p2 - p1) ** 2)
    P = a * b * c
    T = (a + b - c) * (a - b + c) * (-a + b + c)
    return nu * (P ** -1.5 + 0.375 * T * P ** -2.5)


def test_perfect_fcc_matches_infinite_lattice_sums(orc):
    """Counts and energies per particle equal shell sums over the infinite crystal."""
    density, rc, nu = 0.8, 2.5, 0.073
    shell = _fcc_shell(density, rc)
    assert len(shell) == 54
    pairs_pp = len(shell) / 2
    lj_pp = 0.5 * sum(4.0 * (np.dot(p, p) ** -6 - np.dot(p, p) ** -3) for p in shell)
    tri = 0
    atm = 0.0
    for i in range(len(shell)):
        for j in range(i + 1, len(shell)):
            if np.sum((shell[i] - shell[j]) ** 2) <= rc * rc:
                tri += 1
                atm += _atm_poly(np.zeros(3), shell[i], shell[j], nu)
    trip_pp = tri / 3.0
    atm_pp = atm / 3.0
    assert pairs_pp == 27 and trip_pp == 210
    # no lattice distance lies near the cutoff, so rounding cannot flip these counts
    r = np.sort(np.unique(np.round(np.linalg.norm(_fcc_shell(density, 3.0), axis=1), 9)))
    assert not np.any(np.abs(r - rc) < 0.05)

    for n_cells in (5, 6):
        x, box = W.perfect_fcc(n_cells, density)
        n = x.shape[0]
        p = orc.pair_forces(x, box, rc=rc, shift=False)
        t = orc.triplet_forces(x, box, nu=nu, rc=rc)
        assert p.count == pairs_pp * n
        assert t.count == trip_pp * n
        assert p.energy / n == pytest.approx(lj_pp, rel=1e-12)
        assert t.energy / n == pytest.approx(atm_pp, rel=1e-12)
        assert np.abs(p.f).max() < 1e-11 and np.abs(t.f).max() < 1e-12  # inversion symmetry
        assert t.virial == pytest.approx(9.0 * t.energy, rel=1e-12)


def test_energy_shift_counts_pairs(orc):
    x, box = _jittered(seed=4)
    a = orc.pair_forces(x, box, shift=False)
    b = orc.pair_forces(x, box, shift=True)
    urc, _ = orc.lj(2.5 ** 2)
    assert b.energy == pytest.approx(a.energy - a.count * urc, rel=1e-12)
    assert np.array_equal(a.f, b.f)


def test_directsum_counts_without_effective_cutoff(orc):
    """A cluster smaller than the cutoff: every pair and triplet interacts, C(N,2), C(N,3)."""
    rng = np.random.default_rng(8)
    n = 40
    d = rng.normal(size=(n, 3))
    x = 10.0 + 0.9 * d / np.linalg.norm(d, axis=1, keepdims=True) * rng.uniform(0.3, 1.0, (n, 1))
    box = np.array([20.0, 20.0, 20.0])
    assert orc.pair_forces(x, box).count == math.comb(n, 2)
    assert orc.triplet_forces(x, box).count == math.comb(n, 3)
    assert orc.triplet_list(x, box).shape[0] == math.comb(n, 3)


def _image_sum(x, box, rc, nu, orc):
    """Periodic triplet energy as a sum over images: every triangle (i, j+n1 L, k+n2 L) whose
    three edges are within rc counts once.  Independent of minimum-image arithmetic."""
    n = x.shape[0]
    shifts = [np.array(s, dtype=float) * box for s in itertools.product((-1, 0, 1), repeat=3)]
    energy, count = 0.0, 0
    for i, j, k in itertools.combinations(range(n), 3):
        for sj in shifts:
            pj = x[j] + sj
            if np.sum((pj - x[i]) ** 2) > rc * rc:
                continue
            for sk in shifts:
                pk = x[k] + sk
                if np.sum((pk - x[i]) ** 2) > rc * rc or np.sum((pk - pj) ** 2) > rc * rc:
                    continue
                energy += orc.atm_energy(pj - x[i], pk - x[i], nu)
                count += 1
    return energy, count


@pytest.mark.parametrize("length", [6.0, 7.9])
def test_periodic_triplets_match_image_sum(orc, length):
    """Boxes between 2 rc and 3 rc: minimum images that do not close a triangle are
    rejected, exactly as the sum over explicit images says."""
    rng = np.random.default_rng(int(length * 10))
    box = np.full(3, length)
    ring = np.array([[0.1 + q * length / 3.0, 1.0, 1.0] for q in range(3)])  # wraps the box
    x = np.concatenate([ring, rng.uniform(0, length, size=(15, 3))])
    e_img, c_img = _image_sum(x, box, 2.5, 0.3, orc)
    t = orc.triplet_forces(x, box, nu=0.3, rc=2.5)
    assert t.count == c_img
    assert t.energy == pytest.approx(e_img, rel=1e-12, abs=1e-15)
    lst = orc.triplet_list(x, box)
    assert lst.shape[0] == c_img
    assert not any(tuple(r) == (0, 1, 2) for r in lst)  # the ring is not a triplet


def test_subset_mode_equals_full_forces(orc):
    x, box = _jittered(seed=12)
    idx = np.random.default_rng(3).choice(x.shape[0], size=30, replace=False)
    f2, f3 = orc.subset_forces(x, box, idx)
    p = orc.pair_forces(x, box)
    t = orc.triplet_forces(x, box)
    assert np.abs(f2 - p.f[idx]).max() <= 1e-12 * np.abs(p.f).max()
    assert np.abs(f3 - t.f[idx]).max() <= 1e-12 * np.abs(t.f).max()


def test_subset_counts_every_member(orc):
    """Subset mode over every particle visits each pair from both members and each
    triplet from all three: twice the pair count and three times the triplet count of
    the whole-system loops."""
    x, box = _jittered(seed=13)
    idx = np.arange(x.shape[0])
    _, _, (npair, ntrip) = orc.subset_forces(x, box, idx, counts=True)
    assert npair == 2 * orc.pair_forces(x, box).count
    assert ntrip == 3 * orc.triplet_forces(x, box).count


def test_triplet_list_matches_count_and_order(orc):
    x, box = _jittered(n_cells=3, density=0.8, jitter=0.1, seed=21)
    lst = orc.triplet_list(x, box)
    t = orc.triplet_forces(x, box)
    assert lst.shape[0] == t.count
    assert np.all(lst[:, 0] < lst[:, 1]) and np.all(lst[:, 1] < lst[:, 2])
    keys = lst[:, 0].astype(np.int64) * 10 ** 6 + lst[:, 1] * 10 ** 3 + lst[:, 2]
    assert np.all(np.diff(keys) > 0)


def test_cell_index_bounds_and_edges(orc):
    x, box = _jittered(seed=31)
    nc = np.array([4, 3, 5], dtype=np.int32)
    box = np.array([box[0], box[1] * 1.1, box[2] * 0.9])
    cells = orc.cell_index(x, box, nc)
    w = orc.wrap(x, box)
    cx = cells % nc[0]
    cy = (cells // nc[0]) % nc[1]
    cz = cells // (nc[0] * nc[1])
    for dim, c in enumerate((cx, cy, cz)):
        h = box[dim] / nc[dim]
        assert np.all(c >= 0) and np.all(c < nc[dim])
        assert np.all(w[:, dim] >= c * h - 1e-12) and np.all(w[:, dim] <= (c + 1) * h + 1e-12)
    edge = np.array([[-1e-300, 0.0, box[2] - 1e-13], [box[0], 2 * box[1] + 0.5, -box[2]],
                     [box[0] * (1 - 1e-16), -3.0 * box[1], 0.5 * box[2]]])
    ce = orc.cell_index(edge, box, nc)
    we = orc.wrap(edge, box)
    assert np.all(we >= 0.0) and np.all(we <= box)
    assert np.all((ce >= 0) & (ce < nc.prod()))
    assert ce[0] % nc[0] == nc[0] - 1 or we[0, 0] == 0.0  # -tiny wraps to the top cell or to 0


def test_error_paths(orc):
    x, box = _jittered(n_cells=3)
    with pytest.raises(orc.OracleError) as e:
        orc.triplet_forces(x, np.full(3, 4.9))
    assert e.value.code == orc.ERR_BOX_TOO_SMALL
    bad = x.copy()
    bad[3, 1] = np.nan
    with pytest.raises(orc.OracleError) as e:
        orc.pair_forces(bad, box)
    assert e.value.code == orc.ERR_NONFINITE
    with pytest.raises(orc.OracleError) as e:
        orc.respa(x, np.zeros_like(x), box, n_iter=7, k=2)
    assert e.value.code == orc.ERR_NOT_MULTIPLE_OF_K


def test_cutoff_is_inclusive(orc):
    """Pairs and triplets at exactly rc interact: the paper's rule is 'less than or equal to
    the cutoff' for pairs and for all three triplet edges (Sec. 4.2.2, Fig. 2 caption).
    2.5 and its square are exact in binary, so the test is exact."""
    box = np.full(3, 10.0)
    x = np.array([[1.0, 1.0, 1.0], [3.5, 1.0, 1.0], [2.25, 2.0, 1.0]])
    assert orc.pair_forces(x, box, rc=2.5).count == 3
    assert orc.triplet_forces(x, box, rc=2.5).count == 1
    x2 = x.copy()
    x2[1, 0] = np.nextafter(3.5, 4.0)
    assert orc.pair_forces(x2, box, rc=2.5).count == 2
    assert orc.triplet_forces(x2, box, rc=2.5).count == 0
