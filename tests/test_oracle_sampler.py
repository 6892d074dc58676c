"""Pins of the oracle's random-batch sampler: Philox KATs, target law, H."""
import os

import numpy as np
from scipy.stats import chi2

from oracle import rbsampler, lattice

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert rbsampler.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])
        out = rbsampler.philox4x32_10_vec(np.array([v[0]]), v[1], v[2], v[3], v[4], v[5])
        assert tuple(int(o[0]) for o in out) == tuple(v[6:10])


def test_H_closed_form():
    for Lx, Ly, a in [(20, 20, 0.4), (600, 600, 0.1), (60, 35, 0.25)]:
        assert abs(lattice.H_direct(Lx, Ly, a) - lattice.H_poisson(Lx, Ly, a)) < 1e-10 * lattice.H_direct(Lx, Ly, a)
    # value quoted for a 600 x 600 box at alpha = 0.1
    assert abs(lattice.H_direct(600, 600, 0.1) - 1144.91559026) < 1e-7


def test_chain_law_and_acceptance():
    alpha, Lx, Ly = 0.4, 20.0, 14.0
    modes, acc = rbsampler.sample_modes(2024, 0, 60000, alpha, Lx, Ly)
    assert acc > 0.9
    assert not np.any((modes[:, 0] == 0) & (modes[:, 1] == 0))
    r = 9
    mx, my = np.meshgrid(np.arange(-r, r + 1), np.arange(-r, r + 1), indexing="ij")
    keep = ~((mx == 0) & (my == 0))
    mx, my = mx[keep], my[keep]
    h = np.exp(-((2 * np.pi * mx / Lx) ** 2 + (2 * np.pi * my / Ly) ** 2) / (4 * alpha ** 2))
    p = h / lattice.H_direct(Lx, Ly, alpha)
    idx = {(a, b): i for i, (a, b) in enumerate(zip(mx, my))}
    obs = np.zeros(len(mx) + 1)
    for a, b in modes:
        obs[idx.get((a, b), len(mx))] += 1
    exp = np.append(p, 1 - p.sum()) * len(modes)
    use = exp > 20
    stat = np.sum((obs[use] - exp[use]) ** 2 / exp[use]) + \
        (obs[~use].sum() - exp[~use].sum()) ** 2 / exp[~use].sum()
    dof = use.sum()
    # consecutive states of an independence chain are mildly correlated
    # (repeats on rejection); inflate by (1 + rej)/(1 - rej)
    infl = (2 - acc) / acc
    assert stat < infl * chi2.ppf(0.9999, dof)


def test_steps_are_deterministic_and_distinct():
    a, _ = rbsampler.sample_modes(1, 5, 100, 0.1, 600, 600)
    b, _ = rbsampler.sample_modes(1, 5, 100, 0.1, 600, 600)
    c, _ = rbsampler.sample_modes(1, 6, 100, 0.1, 600, 600)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def _chi2_vs_h(modes, alpha, Lx, Ly, r=9):
    mx, my = np.meshgrid(np.arange(-r, r + 1), np.arange(-r, r + 1), indexing="ij")
    keep = ~((mx == 0) & (my == 0))
    mx, my = mx[keep], my[keep]
    h = np.exp(-((2 * np.pi * mx / Lx) ** 2 + (2 * np.pi * my / Ly) ** 2) / (4 * alpha ** 2))
    p = h / lattice.H_direct(Lx, Ly, alpha)
    idx = {(a, b): i for i, (a, b) in enumerate(zip(mx, my))}
    obs = np.zeros(len(mx) + 1)
    for a, b in modes:
        obs[idx.get((int(a), int(b)), len(mx))] += 1
    exp = np.append(p, 1 - p.sum()) * len(modes)
    use = exp > 20
    stat = np.sum((obs[use] - exp[use]) ** 2 / exp[use]) + \
        (obs[~use].sum() - exp[~use].sum()) ** 2 / exp[~use].sum()
    return stat, use.sum()


def test_iid_sampler_law():
    """i.i.d. draws follow h(k)/H over k != 0: chi-square without any
    correlation allowance, never (0, 0)."""
    alpha, Lx, Ly = 0.4, 20.0, 14.0
    modes = rbsampler.sample_modes_iid(77, 3, 60000, alpha, Lx, Ly)
    assert not np.any((modes[:, 0] == 0) & (modes[:, 1] == 0))
    stat, dof = _chi2_vs_h(modes, alpha, Lx, Ly)
    assert stat < chi2.ppf(0.9999, dof)


def test_iid_sampler_marginal_and_tiny_box():
    """The m_x table is the marginal of h over k != 0 (direct lattice sums),
    and a box where (0, 0) would hold almost all of an unconditioned product
    law still yields valid non-zero modes."""
    alpha, Lx, Ly = 0.3, 9.0, 25.0
    cx, cy, cy_nz, mxm, mym = rbsampler.iid_tables(alpha, Lx, Ly)
    H = lattice.H_direct(Lx, Ly, alpha)
    ms = np.arange(-mxm, mxm + 1)
    mys = np.arange(-mym, mym + 1)
    prob = np.diff(np.concatenate([[0.0], cx]))
    for m, pm in zip(ms, prob):
        hm = np.exp(-((2 * np.pi * m / Lx) ** 2 + (2 * np.pi * mys / Ly) ** 2) / (4 * alpha ** 2))
        if m == 0:
            hm = hm[mys != 0]
        assert abs(pm - hm.sum() / H) < 1e-14
    assert cx[-1] == 1.0 and cy[-1] == 1.0 and cy_nz[-1] == 1.0
    modes = rbsampler.sample_modes_iid(5, 0, 2000, 0.05, 12.0, 12.0)
    assert not np.any((modes[:, 0] == 0) & (modes[:, 1] == 0))
    assert np.all(np.abs(modes) <= 1)


def test_iid_sampler_deterministic_and_step_dependent():
    a = rbsampler.sample_modes_iid(1, 5, 100, 0.1, 600, 600)
    b = rbsampler.sample_modes_iid(1, 5, 100, 0.1, 600, 600)
    c = rbsampler.sample_modes_iid(1, 6, 100, 0.1, 600, 600)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
