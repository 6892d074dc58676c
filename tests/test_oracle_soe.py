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


def test_reduced_table(soe_tables):
    """The model-reduced M = 10 table (oracle.soe.reduced_soe, written by
    tests/golden/gen_soe_tables.py): its sup error against the Gaussian itself,
    tail, moments and conjugate pairs -- the accuracy the Talbot rule needs
    M = 16 for, with 10 terms."""
    w, s = soe_tables["r10"]
    assert len(w) == 10
    x = np.linspace(0.0, 8.0, 80001)
    err = np.abs(soe.soe_eval(w, s, x) - np.exp(-x * x)).max()
    assert err < 5e-10
    wt, st = soe_tables[16]
    assert err < np.abs(soe.soe_eval(wt, st, x) - np.exp(-x * x)).max()
    xt = np.linspace(8.0, 400.0, 4001)
    assert np.abs(soe.soe_eval(w, s, xt)).max() < 5e-10
    assert abs(np.sum(w) - 1.0) < 5e-10
    assert abs(np.sum(w / s) - np.sqrt(np.pi) / 2) < 1e-7
    assert np.all(s.real > 0) and np.all(np.abs(s.imag) > 1e-3)
    order = np.argsort(s.imag)
    np.testing.assert_allclose(s[order], np.conj(s[order][::-1]), rtol=1e-14)
    np.testing.assert_allclose(w[order], np.conj(w[order][::-1]), rtol=1e-12)


def test_balanced_truncation_steps():
    """The reduction's steps on a case with a known answer: truncating the
    Talbot table to as many states as it has reproduces its exponents, and the
    Hankel-bound behaviour shows in the unpolished reduced tables (each two
    more states gain at least a factor 30 in sup error)."""
    w0, s0 = soe.talbot_soe(8)
    poles = soe._balanced_truncation_poles(w0, s0, 8)
    assert len(poles) == 8
    for p in poles:
        assert np.abs(s0 - p).min() < 1e-8 * abs(p)
    wr, sr, _ = soe.best_talbot_soe(48)
    errs = []
    for M in (4, 6, 8):
        p = soe._balanced_truncation_poles(wr, sr, M)
        sp = p[p.imag > 0]
        wp = soe._lsq_weights(sp, soe._fit_grid())
        errs.append(soe.sup_error(*soe._pair_table(wp, sp), n=20001))
    for a, b in zip(errs, errs[1:]):
        assert b < a / 30
