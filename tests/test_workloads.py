"""Seeded input generators: shapes, determinism, temperature, density."""
import numpy as np
import pytest

from paper_2507_11172_amd import workloads as W


def test_fcc_shapes_and_box():
    w = W.plain_fp64()
    assert w.x.shape == (500, 3) and w.v.shape == (500, 3)
    assert w.box.shape == (1, 3)
    assert w.box[0, 0] == pytest.approx(8.5499, abs=1e-4)
    assert np.all(w.x >= 0) and np.all(w.x < w.box[0])
    assert w.n_particles.tolist() == [500]


def test_seeded_and_reproducible():
    a, b = W.plain_fp64(), W.plain_fp64()
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)
    c = W.fcc_workload("other", 5, 999)
    assert not np.array_equal(a.x, c.x)


def test_maxwell_boltzmann_exact_temperature():
    v = W.maxwell_boltzmann(4000, 0.7, W.rng_for(3))
    assert np.abs(v.mean(axis=0)).max() < 1e-14
    assert float(np.sum(v * v)) / (3 * 4000 - 3) == pytest.approx(0.7, rel=1e-12)


def test_fcc_subset_density():
    x, box = W.fcc_subset(1234, 0.65, 0.05, W.rng_for(1))
    assert x.shape == (1234, 3)
    assert 1234 / np.prod(box) == pytest.approx(0.65, rel=1e-12)
    d = x[:, None, :] - x[None, :, :]
    d -= box * np.rint(d / box)
    r = np.sqrt(np.sum(d * d, axis=2)) + np.eye(1234) * 9
    assert r.min() > 0.5  # lattice sites stay distinct under jitter


def test_slab_small():
    x, box = W.slab(6000, 0.75, 0.02, W.rng_for(4))
    assert x.shape == (6000, 3)
    assert box[2] == pytest.approx(3 * box[0])
    z = x[:, 2]
    inside = (z >= box[2] / 3) & (z < 2 * box[2] / 3)
    assert inside.sum() == int(round(0.75 * box[0] ** 3))
    assert np.all(x >= 0) and np.all(x < box)


def test_batched_small():
    w = W.batched(n_replicas=6, n_min=200, n_max=600)
    assert w.n_systems == 6
    assert w.x.shape[0] == int(w.n_particles.sum())
    assert np.all(w.n_particles >= 200) and np.all(w.n_particles <= 600)
    off = 0
    for s in range(6):
        n = int(w.n_particles[s])
        xs = w.x[off:off + n]
        assert np.all(xs >= 0) and np.all(xs < w.box[s])
        off += n
