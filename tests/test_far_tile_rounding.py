"""Rounding of the mixed-precision far-tile forms, checked on the host.

The spatially ordered mixed plans take a source tile as "far" from a group of
targets when the gap between their bounding boxes exceeds the tile's own
diagonal; for such tiles the pair separations come from float32 coordinates
relative to the tile's centre c, either subtracted per pair (x_j' - x_i') or
through the expanded squared distance q_j + q_i - 2 x_i'.x_j' with the force
sum taken as sum s_j x_j' - x_i' sum s_j.  The stated bound for the mixed
path is about 10u per pair plus 255u of the tile's sum of |f| (u = 2^-24).

This emulates both forms with numpy float32 arithmetic (a fused multiply-add
as an exact float64 product and sum rounded once to float32; the reciprocal
square root correctly rounded) and checks them against a float64 sum of the
softened pair terms of Eqs. (1)-(2), for tiles of random shape and size,
targets at gaps just above the criterion and far beyond it, translated
systems and zero softening (measured worst case: about 12u for either form).
It also shows the criterion is needed: for targets next to the tile both
forms lose the bound.  The jerk's far-tile form (velocities relative to the
velocity of the tile's first source) is checked the same way on the
kinematics of a rotating disk (measured worst case about 13u).  The
quarter-tile form (far test per wave and per quarter of 64 sources, far
quarters relative to the quarter's centre, near ones float64-formed, one
float32 sum over the tile) is checked on elongated tiles whose quarters fall
on both sides of the criterion."""
import numpy as np
import pytest

U = 2.0 ** -24
T = 256


def f32(v):
    return np.asarray(v, dtype=np.float64).astype(np.float32)


def fma32(a, b, c):
    # exact float32 x float32 product in float64, one rounding of the sum
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def rsq32(r2):
    return (1.0 / np.sqrt(r2.astype(np.float64))).astype(np.float32)


def exact(xs, m, xt, eps2):
    d = xs[None, :, :] - xt[:, None, :]                       # targets x sources x 3
    r2 = (d * d).sum(-1) + eps2
    w = np.where(r2 > 0, m[None, :] / np.where(r2 > 0, r2, 1.0) ** 1.5, 0.0)
    f = (w[:, :, None] * d).sum(1)
    scale = (w * np.sqrt((d * d).sum(-1))).sum(1)             # sum of |f_j|
    return f, scale


def subtracted(xs, m, xt, eps2, c):
    sj = f32(xs - c)
    ti = f32(xt - c)
    e2 = np.float32(eps2)
    acc = np.zeros((xt.shape[0], 3), np.float32)
    for j in range(xs.shape[0]):
        d = sj[j][None, :] - ti                               # float32 subtraction
        r2 = fma32(d[:, 0], d[:, 0], fma32(d[:, 1], d[:, 1], fma32(d[:, 2], d[:, 2], np.full(len(d), e2))))
        y = np.where(r2 > 0, rsq32(np.where(r2 > 0, r2, 1)), np.float32(0))
        sc = (np.float32(m[j]) * y) * (y * y)
        for k in range(3):
            acc[:, k] = fma32(sc, d[:, k], acc[:, k])
    return acc.astype(np.float64)


def expanded(xs, m, xt, eps2, c):
    sj = f32(xs - c)
    qj = f32(((xs - c) ** 2).sum(1))
    dti = xt - c
    w = f32(-2.0 * dti)
    qi = f32((dti ** 2).sum(1) + eps2)
    acc = np.zeros((xt.shape[0], 3), np.float32)
    ssum = np.zeros(xt.shape[0], np.float32)
    for j in range(xs.shape[0]):
        base = (np.float32(qj[j]) + qi).astype(np.float32)
        r2 = fma32(np.full(len(w), sj[j, 0]), w[:, 0],
                   fma32(np.full(len(w), sj[j, 1]), w[:, 1], fma32(np.full(len(w), sj[j, 2]), w[:, 2], base)))
        y = np.where(r2 > 0, rsq32(np.where(r2 > 0, r2, 1)), np.float32(0))
        sc = (np.float32(m[j]) * y) * (y * y)
        for k in range(3):
            acc[:, k] = fma32(sc, np.full(len(sc), sj[j, k]), acc[:, k])
        ssum = (ssum + sc).astype(np.float32)
    # the x_i' sum term in float64, once per tile
    return acc.astype(np.float64) - dti * ssum.astype(np.float64)[:, None]


def tile_and_targets(rng, gap_over_diag, shift, flat):
    ext = np.array([1.0, rng.uniform(0.2, 1.0), 0.05 if flat else rng.uniform(0.2, 1.0)])
    ext = ext * 10.0 ** rng.uniform(-2, 1)
    xs = shift + rng.uniform(-0.5, 0.5, (T, 3)) * ext
    lo, hi = xs.min(0), xs.max(0)
    c = 0.5 * (lo + hi)
    diag = np.linalg.norm(hi - lo)
    # targets on random directions at a given gap from the tile's box
    u = rng.normal(size=(48, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    half = 0.5 * (hi - lo)
    reach = np.abs(u) @ half                                  # box support along u
    xt = c + u * (reach + gap_over_diag * diag)[:, None]
    m = rng.uniform(0.5, 1.5, T) / T
    return xs, m, xt, c, diag


@pytest.mark.parametrize("form", ["subtracted", "expanded"])
@pytest.mark.parametrize("gap_over_diag", [1.05, 2.0, 30.0])
@pytest.mark.parametrize("shift", [0.0, 1.0e3])
def test_far_tile_forms_within_mixed_bound(form, gap_over_diag, shift):
    rng = np.random.default_rng(int(gap_over_diag * 100) + int(shift) + (form == "expanded"))
    fn = subtracted if form == "subtracted" else expanded
    worst = 0.0
    for trial in range(4):
        xs, m, xt, c, diag = tile_and_targets(rng, gap_over_diag, shift, flat=trial % 2 == 0)
        # keep only targets outside the tile's box by more than its diagonal
        lo, hi = xs.min(0), xs.max(0)
        g = np.maximum(0.0, np.maximum(lo - xt, xt - hi))
        far = (g * g).sum(1) > diag * diag
        xt = xt[far]
        if xt.size == 0:
            continue
        for eps2 in (0.0, (0.05 * diag) ** 2):
            f, scale = exact(xs, m, xt, eps2)
            got = fn(xs, m, xt, eps2, c)
            err = np.linalg.norm(got - f, axis=1) / scale
            worst = max(worst, float(err.max()))
    assert worst <= (10 + 255) * U, worst
    # and in practice far below the worst case
    assert worst <= 40 * U, worst


def test_expanded_form_needs_the_far_criterion():
    # targets next to (here among) the tile's sources: the tile-local
    # coordinates are no longer small against the separations, both forms
    # lose the bound (the expanded one by far more, its squared distance
    # cancels), so such tiles take float64-formed separations
    rng = np.random.default_rng(3)
    xs = rng.uniform(-0.5, 0.5, (T, 3))
    m = np.full(T, 1.0 / T)
    c = 0.5 * (xs.min(0) + xs.max(0))
    xt = xs[:8] + 1e-4 * rng.normal(size=(8, 3))             # targets among the sources
    f, scale = exact(xs, m, xt, 0.0)
    err_exp = (np.linalg.norm(expanded(xs, m, xt, 0.0, c) - f, axis=1) / scale).max()
    err_sub = (np.linalg.norm(subtracted(xs, m, xt, 0.0, c) - f, axis=1) / scale).max()
    assert err_sub > (10 + 255) * U, err_sub
    assert err_exp > 100 * err_sub, (err_exp, err_sub)


def jerk_exact(xs, vs, m, xt, vt, eps2):
    d = xs[None, :, :] - xt[:, None, :]
    u = vs[None, :, :] - vt[:, None, :]
    r2 = (d * d).sum(-1) + eps2
    inv3 = m[None, :] / r2 ** 1.5
    rv = (d * u).sum(-1)
    term = inv3[:, :, None] * (u - (3.0 * rv / r2)[:, :, None] * d)
    return term.sum(1), np.linalg.norm(term, axis=-1).sum(1)


def jerk_far(xs, vs, m, xt, vt, eps2, c, w):
    # float32 tile-local positions (about the tile's centre c) and velocities
    # (about the velocity w of the tile's first source), float32 pair terms
    sx, sv = f32(xs - c), f32(vs - w)
    tx, tv = f32(xt - c), f32(vt - w)
    e2 = np.float32(eps2)
    acc = np.zeros((xt.shape[0], 3), np.float32)
    for j in range(xs.shape[0]):
        d = sx[j][None, :] - tx
        u = sv[j][None, :] - tv
        r2 = fma32(d[:, 0], d[:, 0], fma32(d[:, 1], d[:, 1], fma32(d[:, 2], d[:, 2], np.full(len(d), e2))))
        y = rsq32(r2)
        y2 = y * y
        sm = (np.float32(m[j]) * y) * y2
        rv = fma32(d[:, 0], u[:, 0], fma32(d[:, 1], u[:, 1], d[:, 2] * u[:, 2]))
        t = (np.float32(-3.0) * rv) * y2
        for k in range(3):
            acc[:, k] = fma32(sm, fma32(t, d[:, k], u[:, k]), acc[:, k])
    return acc.astype(np.float64)


@pytest.mark.parametrize("gap_over_diag", [1.05, 3.0, 30.0])
def test_far_tile_jerk_on_disk_kinematics(gap_over_diag):
    # a tile of a rotating disk (flat rotation curve plus a 10% dispersion):
    # the tile-local velocities keep the jerk well inside the mixed gate,
    # conditioned by the sum of the pair terms' magnitudes
    rng = np.random.default_rng(int(gap_over_diag * 10))
    worst = 0.0
    for trial in range(3):
        centre = np.array([rng.uniform(1.0, 4.0), 0.0, 0.0])
        xs = centre + rng.uniform(-0.5, 0.5, (T, 3)) * np.array([0.3, 0.3, 0.02])

        def kin(x):
            R = np.hypot(x[:, 0], x[:, 1])
            vrot = np.stack([-x[:, 1] / R, x[:, 0] / R, np.zeros(len(x))], 1)
            return vrot + 0.1 * rng.normal(size=x.shape)

        vs = kin(xs)
        lo, hi = xs.min(0), xs.max(0)
        c, diag, half = 0.5 * (lo + hi), np.linalg.norm(hi - lo), 0.5 * (hi - lo)
        dirs = rng.normal(size=(32, 3)) * np.array([1.0, 1.0, 0.1])
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        xt = c + dirs * ((np.abs(dirs) @ half) + gap_over_diag * diag)[:, None]
        g = np.maximum(0.0, np.maximum(lo - xt, xt - hi))
        xt = xt[(g * g).sum(1) > diag * diag]
        vt = kin(xt)
        m = np.full(T, 1.0 / T)
        eps2 = 0.02 ** 2
        f, scale = jerk_exact(xs, vs, m, xt, vt, eps2)
        got = jerk_far(xs, vs, m, xt, vt, eps2, c, vs[0])
        worst = max(worst, float((np.linalg.norm(got - f, axis=1) / scale).max()))
    assert worst <= 2e-5, worst
    assert worst <= 100 * U, worst


def quarter_tile(xs, m, xt, eps2):
    """The quarter-tile form (jsrc 4) for one wave: the far test per quarter
    of 64 sources against the box of the wave's targets, far quarters
    subtracting float32 coordinates relative to the quarter's centre, near
    quarters rounding float64 differences; all terms into one float32 sum.
    Returns the sum and the number of far quarters."""
    tlo, thi = xt.min(0), xt.max(0)
    e2 = np.float32(eps2)
    acc = np.zeros((xt.shape[0], 3), np.float32)
    nfar = 0
    for q in range(T // 64):
        s = slice(64 * q, 64 * q + 64)
        lo, hi = xs[s].min(0), xs[s].max(0)
        g = np.maximum(0.0, np.maximum(lo - thi, tlo - hi))
        far = (g * g).sum() > ((hi - lo) ** 2).sum()
        nfar += int(far)
        if far:
            c = 0.5 * (lo + hi)
            sj, ti = f32(xs[s] - c), f32(xt - c)
        for j in range(64 * q, 64 * q + 64):
            d = (sj[j - 64 * q][None, :] - ti) if far else f32(xs[j][None, :] - xt)
            r2 = fma32(d[:, 0], d[:, 0], fma32(d[:, 1], d[:, 1], fma32(d[:, 2], d[:, 2], np.full(len(d), e2))))
            y = np.where(r2 > 0, rsq32(np.where(r2 > 0, r2, 1)), np.float32(0))
            sc = (np.float32(m[j]) * y) * (y * y)
            for k in range(3):
                acc[:, k] = fma32(sc, d[:, k], acc[:, k])
    return acc.astype(np.float64), nfar


@pytest.mark.parametrize("shift", [0.0, 1.0e3])
def test_quarter_tile_form_within_mixed_bound(shift):
    # an elongated tile whose quarters follow one another along x (as along a
    # space-filling curve) and a wave's 64 targets in a clump near one end:
    # quarters far from the clump take the quarter-local form, the others
    # float64-formed separations; the tile's float32 sum stays inside the
    # mixed bound, and both kinds of quarter occur
    rng = np.random.default_rng(7 + int(shift))
    worst, nfars = 0.0, []
    for trial in range(6):
        length = rng.uniform(4.0, 8.0)
        xs = rng.uniform(0.0, 1.0, (T, 3)) * np.array([length, 1.0, rng.uniform(0.05, 1.0)])
        xs = xs[np.argsort(xs[:, 0], kind="stable")] + shift
        m = rng.uniform(0.5, 1.5, T) / T
        xt = xs[rng.integers(0, 16)] + rng.normal(size=(64, 3)) * 0.05
        for eps2 in (0.0, 1e-4):
            got, nfar = quarter_tile(xs, m, xt, eps2)
            f, scale = exact(xs, m, xt, eps2)
            err = np.linalg.norm(got - f, axis=1) / scale
            worst = max(worst, float(err.max()))
            nfars.append(nfar)
    assert worst <= (10 + 255) * U, worst
    assert worst <= 40 * U, worst
    assert 0 < min(nfars) and max(nfars) < 4, nfars
