"""Pins of the oracle's SOE tables: sup-norm error and exact moments."""
import numpy as np
import pytest

from oracle import soe

EPS = {8: 4e-5, 12: 2e-7, 16: 1e-9, 20: 5e-12, 24: 5e-14}


@pytest.mark.parametrize("M", [8, 12, 16, 20, 24])
def test_table_sup_error(soe_tables, M):
    w, s = soe_tables[M]
    assert len(w) == M
    x = np.linspace(0.0, 8.0, 80001)
    err = np.abs(soe.soe_eval(w, s, x) - np.exp(-x * x)).max()
    assert err < EPS[M]
    # far tail: SOE must stay below eps where the Gaussian vanishes
    xt = np.linspace(8.0, 400.0, 4001)
    assert np.abs(soe.soe_eval(w, s, xt)).max() < EPS[M]


@pytest.mark.parametrize("M", [8, 16, 24])
def test_table_moments_and_symmetry(soe_tables, M):
    w, s = soe_tables[M]
    # value at 0: sum w = 1; integral over [0, inf): sum w/s = sqrt(pi)/2;
    # slope at 0+: -sum w s = d/dx e^{-x^2} at 0 = 0
    assert abs(np.sum(w) - 1.0) < EPS[M]
    assert abs(np.sum(w / s) - np.sqrt(np.pi) / 2) < 200 * EPS[M]
    assert abs(np.sum(w * s)) < 50 * EPS[M]
    assert np.all(s.real > 0)
    # conjugate-closed, with no real node
    order = np.argsort(s.imag)
    np.testing.assert_allclose(s[order], np.conj(s[order][::-1]), rtol=1e-14)
    np.testing.assert_allclose(w[order], np.conj(w[order][::-1]), rtol=1e-12)
    assert np.all(np.abs(s.imag) > 1e-3)


def test_talbot_converges_geometrically():
    errs = [soe.sup_error(*soe.talbot_soe(M), n=20001) for M in (8, 12, 16, 20)]
    for a, b in zip(errs, errs[1:]):
        assert b < a / 50
