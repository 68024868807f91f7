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
