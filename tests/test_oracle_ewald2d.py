"""Pins of O1 (exact Ewald2D) against values fixed by the physics, not by O1."""
import mpmath
import numpy as np
import pytest

import workloads as wl
from oracle import ewald2d, lattice


def madelung_square():
    # M2 = 4 (sqrt 2 - 1)(-zeta(1/2)) beta(1/2): 2-D square ionic lattice (textbook)
    mpmath.mp.dps = 30
    beta_half = mpmath.dirichlet(0.5, [0, 1, 0, -1])
    return float(4 * (mpmath.sqrt(2) - 1) * (-mpmath.zeta(0.5)) * beta_half)


def test_madelung_constant_value():
    assert abs(madelung_square() - 1.6155426267128247) < 1e-15


@pytest.mark.parametrize("alpha", [1.1, 2.3])
def test_square_ionic_lattice(alpha):
    a = 1.3
    pos, q = wl.square_ionic_cell(a, 0.7)
    r = ewald2d.ewald2d(pos, q, (2 * a, 2 * a, 2.0), alpha, rc=10.0, kc=14 * alpha)
    M2 = madelung_square()
    np.testing.assert_allclose(r["phi"], -q * M2 / a, rtol=1e-12, atol=0)
    assert abs(r["U"] - (-2 * M2 / a)) < 1e-12
    np.testing.assert_allclose(r["F"], 0.0, atol=1e-12)


def test_alpha_independence():
    box = (5.0, 6.0, 3.0)
    pos, q = wl.random_system(8, box, seed=1)
    rs = [ewald2d.ewald2d(pos, q, box, a, rc=7 / a, kc=14 * a) for a in (0.8, 1.3, 1.8)]
    for r in rs[1:]:
        assert abs(r["U"] - rs[0]["U"]) < 1e-12 * abs(rs[0]["U"]) + 1e-13
        np.testing.assert_allclose(r["phi"], rs[0]["phi"], rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(r["F"], rs[0]["F"], rtol=1e-10, atol=1e-11)


def test_brute_force_lattice_sum():
    box = (5.0, 6.0, 3.0)
    pos, q = wl.random_system(4, box, seed=3)
    r = ewald2d.ewald2d(pos, q, box, 1.0, rc=7.0, kc=14.0)
    Rs = [200, 300, 450, 700, 1000]
    U = lattice.extrapolate(Rs, [lattice.direct_energy(pos, q, box, R) for R in Rs], order=4)
    assert abs(U - r["U"]) < 1e-7 * abs(r["U"])
    Rs = [100, 150, 220, 330, 500]
    Fs = [lattice.direct_forces(pos, q, box, R) for R in Rs]
    F = np.array([[lattice.extrapolate(Rs, [f[i, c] for f in Fs], order=4) for c in range(3)]
                  for i in range(4)])
    np.testing.assert_allclose(F, r["F"], atol=1e-5 * np.abs(r["F"]).max())


def test_force_is_minus_gradient():
    box = (5.0, 6.0, 3.0)
    pos, q = wl.random_system(6, box, seed=7)
    alpha, rc, kc = 1.2, 6.0, 17.0
    r = ewald2d.ewald2d(pos, q, box, alpha, rc, kc)
    h = 1e-5
    for i in (0, 3):
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, c] += h
            pm[i, c] -= h
            d = (ewald2d.ewald2d(pp, q, box, alpha, rc, kc)["U"]
                 - ewald2d.ewald2d(pm, q, box, alpha, rc, kc)["U"]) / (2 * h)
            assert abs(-d - r["F"][i, c]) < 1e-7


def test_xi_even_and_smooth_at_zero():
    # d/dz (xi+ + xi-) = k (xi+ - xi-) vanishes at z = 0 (even, smooth kernel)
    for k in (0.3, 1.7, 6.0):
        G, Gd = ewald2d.xi_sum(k, np.array([0.0]), 0.9)
        assert abs(Gd[0]) < 1e-15
        h = 1e-6
        Gp, _ = ewald2d.xi_sum(k, np.array([h]), 0.9)
        Gm, _ = ewald2d.xi_sum(k, np.array([2 * h]), 0.9)
        assert abs((Gm - Gp)[0] / h - k * ewald2d.xi_sum(k, np.array([1.5 * h]), 0.9)[1][0]) < 1e-6
