"""Host-side measures of the long-run driver: the map comparison and the
m = 2 (bar / two-armed) amplitude, on hand-made maps."""
import numpy as np
import pytest


def test_m2_amplitude_of_point_symmetric_pair():
    from paper_1803_01190_amd import longrun as lr
    grid = lr.Grid(64, 64, -4.0, -4.0, 0.125)
    a = np.zeros((64, 64), dtype=np.uint32)
    a[32, 40] = 10          # cell centre (1.0625, 0.0625)
    a[31, 23] = 10          # its mirror through the origin: a pure m = 2 pattern
    assert lr.nonaxisymmetry(a, grid) == pytest.approx(1.0, rel=1e-12)
    ring = np.zeros((64, 64), dtype=np.uint32)
    for (iy, ix) in ((32, 40), (31, 23), (40, 31), (23, 32)):   # four-fold symmetric: no m = 2
        ring[iy, ix] = 10
    assert lr.nonaxisymmetry(ring, grid) <= 1e-12
    assert lr.nonaxisymmetry(np.zeros((64, 64), dtype=np.uint32), grid) == 0.0


def test_compare_maps():
    from paper_1803_01190_amd import longrun as lr
    a = np.zeros((8, 8), dtype=np.uint32)
    a[4, 4] = 10
    a[2, 3] = 10
    b = a.copy()
    b[4, 4] = 5
    b[5, 4] = 5             # half of one clump moved by a cell
    c = lr.compare_maps(a, b)
    assert c["l1_frac"] == pytest.approx(10 / 20) and c["max_frac"] == pytest.approx(5 / 10)
    assert lr.compare_maps(a, a) == {"l1_frac": 0.0, "max_frac": 0.0}


def test_record_deviations_table_and_round_trip(tmp_path):
    # the Table 2 quantities are the largest deviations from the first sample:
    # |P - P0|, |Lz - Lz0| / |Lz0|, |E - E0| / |E0|, |com - com0|; a saved
    # record (the long-run pieces resume from it) loads back unchanged
    from paper_1803_01190_amd import longrun as lr
    rec = lr.Record()
    samples = [(0, -2.0, (0.0, 0.0, 0.0), 4.0, (0.0, 0.0, 0.0)),
               (50, -2.002, (3e-3, 4e-3, 0.0), 4.0 + 8e-3, (0.0, 1e-2, 0.0)),
               (100, -1.999, (0.0, 0.0, 1e-3), 4.0 - 4e-3, (2e-3, 0.0, 0.0))]
    for step, E, P, Lz, C in samples:
        rec.add(step, {"E": E, "Px": P[0], "Py": P[1], "Pz": P[2], "Lz": Lz, "Cx": C[0], "Cy": C[1], "Cz": C[2]})
    t = rec.table2()
    assert t["dP_abs_max"] == pytest.approx(5e-3)
    assert t["dL_rel_max"] == pytest.approx(2e-3)
    assert t["dE_rel_max"] == pytest.approx(1e-3)
    assert t["dcom_abs_max"] == pytest.approx(1e-2)
    rec.maps = {0: np.arange(12, dtype=np.uint32).reshape(3, 4), 100: np.ones((3, 4), dtype=np.uint32)}
    rec.busy_s, rec.evals = 1.5, 100
    stem = str(tmp_path / "rec")
    rec.save(stem)
    back = lr.Record.load(stem)
    assert back.steps == rec.steps and back.E == rec.E and back.Lz == rec.Lz
    assert back.P == rec.P and back.com == rec.com
    assert back.busy_s == rec.busy_s and back.evals == rec.evals
    assert sorted(back.maps) == [0, 100]
    for k in rec.maps:
        assert np.array_equal(back.maps[k], rec.maps[k])
    assert lr.interactions_per_s(1000, back) == pytest.approx(100 * 1e6 / 1.5)
