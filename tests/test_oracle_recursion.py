"""Pin of O3 (the plain O(N) recursion): equal to the O2 pair sums to rounding."""
import numpy as np
import pytest

import workloads as wl
from oracle import soewald2d, lattice, rbsampler
from oracle import recursion as o3


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_o3_equals_o2_exact_k(soe_tables):
    w, s = soe_tables[16]
    c = wl.make_config(1)
    box, pos, q, alpha, kc = c["box"], c["pos"], c["q"], c["alpha"], c["kc"]
    m, wt = soewald2d.exact_modes(box[0], box[1], alpha, kc)
    r2 = soewald2d.long_range(pos, q, box, alpha, w, s, m, wt)
    r3 = o3.long_range(pos, q, box, alpha, w, s, m, wt)
    assert _rel(r3["phi"], r2["phi"]) < 1e-12
    assert _rel(r3["F"], r2["F"]) < 1e-12
    assert abs(r3["U"] - r2["U"]) < 1e-12 * abs(r2["U"])


def test_o3_equals_o2_random_batch(soe_tables):
    w, s = soe_tables[24]
    box = (60.0, 60.0, 10.0)
    pos, q = wl.random_system(400, box, seed=4)
    alpha = 0.25
    H = lattice.H_direct(box[0], box[1], alpha)
    modes, _ = rbsampler.sample_modes(7, 3, 20, alpha, box[0], box[1])
    D = soewald2d.diag_constant(box[0], box[1], alpha, w, s)
    wt = soewald2d.rb_weights(20, H, box[0], box[1])
    r2 = soewald2d.long_range(pos, q, box, alpha, w, s, modes, wt, include_self_pair=False, diag=D)
    r3 = o3.long_range(pos, q, box, alpha, w, s, modes, wt, include_self_pair=False, diag=D,
                       nthreads=2)
    assert _rel(r3["phi"], r2["phi"]) < 1e-11
    assert _rel(r3["F"], r2["F"]) < 1e-11


def test_o3_ties_and_degenerate(soe_tables):
    w, s = soe_tables[16]
    box = (8.0, 8.0, 2.0)
    # many equal z (sort ties): the z-force of a tied pair differs between
    # sgn = 0 (O2) and the sort order (O3) only by K'(0) terms, which vanish
    # for k != 0 and are ~ sum(w s) for k = 0.
    pos, q = wl.random_system(40, box, seed=8, z_values=[0.5, 1.0, 1.5])
    alpha, kc = 0.8, 5.0
    m, wt = soewald2d.exact_modes(box[0], box[1], alpha, kc)
    r2 = soewald2d.long_range(pos, q, box, alpha, w, s, m, wt)
    r3 = o3.long_range(pos, q, box, alpha, w, s, m, wt)
    assert _rel(r3["phi"], r2["phi"]) < 1e-11
    assert np.abs(r3["F"] - r2["F"]).max() < 1e-7
    # empty mode list and single particle
    p1, q1 = pos[:1], np.zeros(1)
    r = o3.long_range(p1, q1, box, alpha, w, s, np.zeros((0, 2), int), np.zeros(0))
    assert r["phi"][0] == 0.0 and np.all(r["F"] == 0.0)
