"""Short-horizon GPU runs of the study runners behind the aluminium experiments (Sec.
4.2.2): the records are finite and shaped as documented, and the cheap invariants hold."""
import math

import pytest

pytestmark = pytest.mark.gpu


def test_al_energy_study_short():
    import bench
    r = bench.al_energy_study(24, [2, 12], "fp64")
    f = r["factors"]
    assert set(f) == {"1", "2", "12"}
    assert f["1"]["mean_rel_dev_vs_sv"] == 0.0
    for q in f.values():
        assert math.isfinite(q["mean_total_energy"]) and len(q["hist"]) == 50
    assert abs(sum(f["12"]["hist"]) - 1.0) < 1e-12


def test_al_pbc_study_short():
    import bench
    r = bench.al_pbc_study(120, 24, [1, 2], "fp64")
    runs = r["runs"]
    assert set(runs) == {"two-body", "k=1", "k=2"}
    assert runs["k=1"]["rdf_l1_vs_sv"] == 0.0
    for q in runs.values():
        assert math.isfinite(q["pressure_mean"]) and len(q["rdf"]) == 100
        # a dense fluid or lattice: the first peak between the LJ minimum and the lattice
        # spacing of the initial state (1.29)
        assert 0.9 < q["rdf_first_peak"][0] < 1.45 and q["rdf_first_peak"][1] > 1.5
    assert runs["k=2"]["samples"] == 60 and runs["k=1"]["samples"] == 120
