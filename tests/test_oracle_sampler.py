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
