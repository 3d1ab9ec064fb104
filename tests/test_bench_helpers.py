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
