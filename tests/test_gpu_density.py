"""GPU surface-density map (nbody_surface_density) against the oracle:
integer counts, so bit-exact, at ragged and full sizes, with off-grid and
NaN particles and the argument checks."""
import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu


def gpu_map(nb, ctx, ic, *grid):
    s = nb.System.from_arrays(ic)
    out = nb.nbody_surface_density(ctx, s, *grid)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("n", [0, 1, 255, 257, 4099, 1 << 17])
def test_disk_map_exact(nb, ctx, orc, n):
    print(f"[case] density disk n={n}", flush=True)
    ic = wl.exp_disk(n, 40 + n % 7)
    grid = (256, 192, -4.5, -3.5, 256 / 9.0, 192 / 7.0)
    got = gpu_map(nb, ctx, ic, *grid)
    ref = orc.surface_density(ic["x"], ic["y"], *grid)
    assert np.array_equal(got, ref)
    assert int(got.sum()) == int(ref.sum())


def test_full_size_disk_and_fine_grid(nb, ctx, orc):
    print("[case] density disk n=2^20, 2048 x 2048", flush=True)
    ic = wl.exp_disk(1 << 20, 2)
    grid = (2048, 2048, -4.0, -4.0, 256.0, 256.0)
    got = gpu_map(nb, ctx, ic, *grid)
    ref = orc.surface_density(ic["x"], ic["y"], *grid)
    assert np.array_equal(got, ref)


def test_off_grid_nan_and_edges(nb, ctx, orc):
    print("[case] density edges", flush=True)
    ic = wl.plummer(3000, 41)
    x, y = ic["x"].copy(), ic["y"].copy()
    x[:10] = np.nan
    y[10:20] = np.inf
    x[20:30] = -1.0          # exactly on the left edge: counted
    x[30:40] = 1.0           # exactly on the right edge: off the grid
    y[40:50] = np.nextafter(1.0, 0.0)
    ic = dict(ic, x=x, y=y)
    grid = (64, 48, -1.0, -1.0, 32.0, 24.0)
    got = gpu_map(nb, ctx, ic, *grid)
    ref = orc.surface_density(x, y, *grid)
    assert np.array_equal(got, ref)
    assert got[:, 0].sum() >= 10


def test_repeat_overwrites(nb, ctx, orc):
    ic = wl.plummer(5000, 42)
    s = nb.System.from_arrays(ic)
    out = torch.full((32, 32), 7, dtype=torch.int32, device="cuda")
    for _ in range(2):
        nb.nbody_surface_density(ctx, s, 32, 32, -2.0, -2.0, 8.0, 8.0, out=out)
    torch.cuda.synchronize()
    ref = orc.surface_density(ic["x"], ic["y"], 32, 32, -2.0, -2.0, 8.0, 8.0)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), ref)


def test_argument_checks(nb, ctx):
    s = nb.System.from_arrays(wl.plummer(10, 1))
    out = torch.zeros(16, dtype=torch.int32, device="cuda")
    for bad in ((0, 16, 0.0, 0.0, 1.0, 1.0), (16, 0, 0.0, 0.0, 1.0, 1.0), (4, 4, 0.0, 0.0, 0.0, 1.0),
                (4, 4, 0.0, 0.0, 1.0, float("nan")), (4, 4, float("inf"), 0.0, 1.0, 1.0),
                (4, 4, 0.0, 0.0, -1.0, 1.0), (1 << 14, 1 << 13, 0.0, 0.0, 1.0, 1.0)):
        with pytest.raises(nb.NBodyError) as ei:
            nb._check(ctx, nb._lib.nbody_surface_density(ctx, nb.ctypes.byref(s.c()), bad[0], bad[1], *bad[2:],
                                                          nb.ctypes.c_void_p(out.data_ptr()), None))
        assert ei.value.status == nb.NB_EINVAL
