"""The host arithmetic of the library's equilibrium-disk iteration
(paper_1803_01190_amd/equilibrium.py: the layer of Eq. (4) for many radial
bins at once, its columns and midplane densities) against the oracle's plain
reference (oracle/equilibrium.py), which is pinned on the isothermal sheet."""
import math

import numpy as np
import pytest


def test_layers_match_oracle():
    from oracle import equilibrium as orc_eq
    from paper_1803_01190_amd import equilibrium as eq
    rho0 = np.array([2.0, 0.5, 0.05, 1.0, 1.0])
    cz2 = np.array([0.3, 0.1, 0.01, 0.2, 0.2])
    rstar = np.array([0.0, 0.1, -0.02, 0.3, -0.4])
    z = np.linspace(0.0, 0.6, 6001)
    prof = eq._layer(rho0, cz2, rstar, 1.0, z)
    for b in range(rho0.size):
        zs, rs = orc_eq.vertical_profile(rho0[b], cz2[b], rstar[b], 1.0, zmax=0.6, h=z[1] - z[0])
        k = min(len(rs), z.size)
        np.testing.assert_allclose(prof[:k, b], rs[:k], rtol=1e-9, atol=1e-12 * rho0[b])
        # beyond the end of the oracle's layer the library's is empty
        assert not prof[len(rs):, b].any()


def test_midplane_density_matches_oracle():
    from oracle import equilibrium as orc_eq
    from paper_1803_01190_amd import equilibrium as eq
    sigma = np.array([0.3, 0.05, 0.01])
    cz2 = math.pi * sigma * 0.1   # sheets of thickness 0.1
    rstar = np.array([0.05, -0.01, 0.0])
    z = np.linspace(0.0, 1.2, 2401)
    got = eq._midplane(sigma, cz2, rstar, 1.0, z)
    for b in range(sigma.size):
        want = orc_eq.solve_rho0(sigma[b], cz2[b], rstar[b], 1.0, zmax=1.2, h=z[1] - z[0])
        assert abs(got[b] - want) <= 1e-6 * want, (b, got[b], want)
    # the sheet's closed form when rho_* = 0
    assert abs(got[2] - math.pi * sigma[2] ** 2 / (2.0 * cz2[2])) <= 1e-4 * got[2]
