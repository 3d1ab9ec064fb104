"""Host-side analysis helpers of the study runners (no GPU)."""
import numpy as np


def test_rdf_of_uniform_points_is_one():
    """Uniform random points in a periodic box: g(r) = 1 up to counting noise, so the shell
    normalisation of the study's RDF is right."""
    import math
    import bench
    rng = np.random.default_rng(5)
    box = np.full(3, 12.0)
    n = 3000
    x = rng.uniform(0.0, 12.0, size=(n, 3))
    r_max, nbins = 5.0, 50
    counts = bench._rdf(x, box, r_max, nbins)
    edges = np.linspace(0.0, r_max, nbins + 1)
    shell = 4.0 / 3.0 * math.pi * np.diff(edges ** 3)
    g = 2.0 * counts / (n * (n / box.prod()) * shell)
    assert counts.sum() > 0
    assert np.abs(g[10:] - 1.0).max() < 0.05   # r > 1: thousands of pairs per shell
    assert abs(np.mean(g[10:]) - 1.0) < 0.01


def test_rdf_counts_each_pair_once_with_minimum_image():
    import bench
    box = np.full(3, 10.0)
    x = np.array([[0.5, 0.5, 0.5], [9.5, 0.5, 0.5], [5.0, 5.0, 5.0]])  # 1.0 apart through the face
    c = bench._rdf(x, box, 2.0, 4)
    assert c.tolist() == [0.0, 0.0, 1.0, 0.0]


def test_bench_rvite_matches_the_oracle_definition():
    """The bench's per-system RVITE (and drift) from energy records equal Eq. 4 as the
    oracle states it, on synthetic records of two systems."""
    import bench
    import oracle
    rng = np.random.default_rng(3)
    rows, nsys = 21, 2
    en = np.zeros((rows, nsys, 5))
    en[:, :, 0] = 50.0 + rng.normal(0.0, 1.0, (rows, nsys))      # K
    en[:, :, 1] = -200.0 + rng.normal(0.0, 1.0, (rows, nsys))    # U2
    en[:, :, 2] = 3.0 + rng.normal(0.0, 0.1, (rows, nsys))       # U3
    n_particles = np.array([100, 300])
    drift, rvite = bench._drift_stats(en, n_particles)
    tot = en[:, :, 0] + en[:, :, 1] + en[:, :, 2]
    ref = [oracle.rvite(tot[:, q], en[:, q, 0]) for q in range(nsys)]
    assert abs(rvite - np.mean(ref)) <= 1e-15 * abs(np.mean(ref))
    ref_drift = np.mean(np.abs(tot[-1] - tot[0]) / n_particles)
    assert abs(drift - ref_drift) <= 1e-15 * abs(ref_drift)
