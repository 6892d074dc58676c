"""Pins of O2 (direct SOE pair sums)."""
import numpy as np
import pytest
from scipy.special import erf

import workloads as wl
from oracle import ewald2d, soewald2d, soe, lattice, rbsampler


def _eps(w, s):
    return soe.sup_error(w, s, n=40001)


@pytest.mark.parametrize("M", [8, 16])
def test_k_kernel_within_thm32_bound(soe_tables, M):
    w, s = soe_tables[M]
    eps = _eps(w, s)
    alpha = 0.7
    z = np.linspace(0.0, 12.0, 2001)
    for k in (0.05, 0.4, 1.3, 3.0, 6.0):
        K, Kd = soewald2d.kernel_k(k, z, alpha, w, s)
        g = np.exp(-k * k / (4 * alpha * alpha))
        G, Gd = ewald2d.xi_sum(k, z, alpha)
        # |xi - xi_M| <= 2 a e^{-k^2/4a^2} eps/(sqrt(pi) k) each (Thm 3.2)
        bound = 2 * 2 * alpha * g * eps / (np.sqrt(np.pi) * k) / k
        assert np.abs(g * K - G / k).max() <= bound * 1.01 + 1e-300
        # |d xi - d xi_M| <= 4 a e^{-k^2/4a^2} eps/sqrt(pi) each
        dbound = 2 * 4 * alpha * g * eps / np.sqrt(np.pi) / k
        assert np.abs(g * Kd - Gd).max() <= dbound * 1.01 + 1e-300


@pytest.mark.parametrize("M", [8, 16])
def test_k0_kernel_within_erf_bound(soe_tables, M):
    w, s = soe_tables[M]
    eps = _eps(w, s)
    alpha, Lz = 0.6, 10.0
    z = np.linspace(0.0, Lz, 2001)
    K0, K0d = soewald2d.kernel_0(z, alpha, w, s)
    exact = z * erf(alpha * z) + np.exp(-(alpha * z) ** 2) / (alpha * np.sqrt(np.pi))
    # erf error <= 2 a z eps/sqrt(pi) (eq. erfSOE), Gaussian error <= eps
    bound = z * 2 * alpha * z * eps / np.sqrt(np.pi) + eps / (alpha * np.sqrt(np.pi))
    assert np.all(np.abs(K0 - exact) <= bound * 1.01 + 1e-15)
    assert np.abs(K0d - erf(alpha * z)).max() < 100 * eps * (1 + alpha * Lz)


def test_kernel_derivative_vanishes_at_zero(soe_tables):
    w, s = soe_tables[16]
    for k in (0.01, 0.5, 2.0):
        K, Kd = soewald2d.kernel_k(k, np.array([0.0]), 0.4, w, s)
        assert abs(Kd[0]) < 1e-13 * (1 + abs(K[0]))


def test_o2_converges_to_exact_ewald(soe_tables):
    c = wl.make_config(1)
    box, pos, q, alpha, kc = c["box"], c["pos"], c["q"], c["alpha"], c["kc"]
    ex = ewald2d.long_range(pos, q, box, alpha, kc)
    prev = None
    for M in (8, 12, 16, 20, 24):
        w, s = soe_tables[M]
        r = soewald2d.exact_k(pos, q, box, alpha, kc, w, s)
        d = max(abs(r["U"] - ex["U"]), np.abs(r["F"] - ex["F"]).max())
        assert d < 10 * _eps(w, s) * np.abs(ex["F"]).max() + 1e-13
        if prev is not None:
            assert d < prev
        prev = d


def test_o2_matches_literal_pair_loop(soe_tables):
    w, s = soe_tables[12]
    box = (7.0, 5.0, 4.0)
    pos, q = wl.random_system(5, box, seed=11)
    alpha, kc = 0.9, 4.0
    modes, wts = soewald2d.exact_modes(box[0], box[1], alpha, kc)
    A = box[0] * box[1]
    phi = np.zeros(5)
    F = np.zeros((5, 3))
    for i in range(5):
        for j in range(5):
            dz = pos[i, 2] - pos[j, 2]
            K0, K0d = soewald2d.kernel_0(np.array([dz]), alpha, w, s)
            phi[i] += -(2 * np.pi / A) * q[j] * K0[0]
            if j != i:
                F[i, 2] += (2 * np.pi / A) * q[i] * q[j] * np.sign(dz) * K0d[0]
            for (mx, my), om in zip(modes, wts):
                kx, ky, k = soewald2d.mode_k(mx, my, box[0], box[1])
                K, Kd = soewald2d.kernel_k(k, np.array([dz]), alpha, w, s)
                th = kx * (pos[i, 0] - pos[j, 0]) + ky * (pos[i, 1] - pos[j, 1])
                phi[i] += om * q[j] * np.cos(th) * K[0]
                if j != i:
                    F[i, 0] += om * q[i] * q[j] * kx * np.sin(th) * K[0]
                    F[i, 1] += om * q[i] * q[j] * ky * np.sin(th) * K[0]
                    F[i, 2] += -om * q[i] * q[j] * np.cos(th) * np.sign(dz) * Kd[0]
        phi[i] -= 2 * alpha * q[i] / np.sqrt(np.pi)
    r = soewald2d.exact_k(pos, q, box, alpha, kc, w, s)
    np.testing.assert_allclose(r["phi"], phi, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(r["F"], F, rtol=1e-11, atol=1e-13)


def test_o2_force_is_minus_gradient(soe_tables):
    w, s = soe_tables[16]
    box = (6.0, 5.0, 3.0)
    pos, q = wl.random_system(6, box, seed=5)
    alpha, kc = 1.0, 7.0

    def U(p):
        return soewald2d.exact_k(p, q, box, alpha, kc, w, s)["U"]

    r = soewald2d.exact_k(pos, q, box, alpha, kc, w, s)
    h = 1e-5
    for i in (1, 4):
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, c] += h
            pm[i, c] -= h
            assert abs(-(U(pp) - U(pm)) / (2 * h) - r["F"][i, c]) < 1e-8


def test_rb_estimator_unbiased(soe_tables):
    """Mean of random-batch energies -> the full k-sum, within the Prop 4.1 band."""
    w, s = soe_tables[12]
    box = (10.0, 10.0, 3.0)
    pos, q = wl.random_system(12, box, seed=21)
    alpha = 0.5
    H = lattice.H_direct(box[0], box[1], alpha)
    D = soewald2d.diag_constant(box[0], box[1], alpha, w, s)
    modes, wts = soewald2d.exact_modes(box[0], box[1], alpha, 2 * alpha * np.sqrt(np.log(1e18)))
    # exact sum over all k != 0 (pairs only) and per-mode contributions f(k)
    f = np.array([soewald2d.long_range(pos, q, box, alpha, w, s, [m], [1.0],
                                       include_self_pair=False, k0=False)["U"] for m in modes])
    _, _, k = soewald2d.mode_k(modes[:, 0], modes[:, 1], box[0], box[1])
    g = np.exp(-k * k / (4 * alpha * alpha))
    A = box[0] * box[1]
    exact = float(np.sum(np.pi / A * g * f))
    # i.i.d. variance of one RB draw of P modes (Prop 4.1, eq. Exi)
    P = 8
    var1 = (H * np.sum(g * (np.pi / A * f) ** 2) - exact ** 2) / P
    R = 300
    vals = []
    for step in range(R):
        m, _ = rbsampler.sample_modes(99, step, P, alpha, box[0], box[1])
        r = soewald2d.long_range(pos, q, box, alpha, w, s, m,
                                 soewald2d.rb_weights(P, H, box[0], box[1]),
                                 include_self_pair=False, k0=False)
        vals.append(r["U"])
    mean = np.mean(vals)
    assert abs(mean - exact) < 5 * np.sqrt(1.5 * var1 / R)
    # and the sample variance matches Prop 4.1 within a loose factor
    assert 0.5 * var1 < np.var(vals) < 2.0 * var1
    assert D > 0


def _diag_exact(Lx, Ly, alpha, tol=1e-18):
    """(pi/A) sum_{k != 0} 2 erfc(k/(2 alpha))/k: the j = i term of phi^k
    (Sec. 2.2, eq. philk at rho_ij = 0, z_ij = 0, where xi^+ + xi^- = 2 erfc(k/2a)),
    summed over the whole lattice with the exact (non-SOE) kernel."""
    from scipy.special import erfc
    kc = 2 * alpha * np.sqrt(-np.log(tol))
    m = ewald2d.kmodes_full(Lx, Ly, kc)
    _, _, k = soewald2d.mode_k(m[:, 0], m[:, 1], Lx, Ly)
    return np.pi / (Lx * Ly) * float(np.sum(2 * erfc(k / (2 * alpha)) / k)), k


@pytest.mark.parametrize("box,alpha", [((20.0, 20.0), 0.4), ((60.0, 35.0), 0.25)])
@pytest.mark.parametrize("M", [8, 16, 24])
def test_diag_constant_is_the_j_eq_i_term(soe_tables, box, alpha, M):
    """The random-batch j = i constant D against the configuration-independent
    j = i term of U^k summed over k != 0 with the exact kernel (Sec. 3.2: the
    constant Q pi erfc(k/2a)/(kA) of the rearranged pair sum): their gap must lie
    within the Thm 3.2 kernel bound summed over the lattice."""
    w, s = soe_tables[M]
    eps = _eps(w, s)
    Lx, Ly = box
    D = soewald2d.diag_constant(Lx, Ly, alpha, w, s)
    Dx, k = _diag_exact(Lx, Ly, alpha)
    g = np.exp(-k * k / (4 * alpha * alpha))
    # Thm 3.2: |g K_k(0) - (xi^+ + xi^-)(k, 0)/k| <= 2 (2 a g eps / (sqrt(pi) k)) / k
    bound = np.pi / (Lx * Ly) * float(np.sum(4 * alpha * g * eps / (np.sqrt(np.pi) * k * k)))
    print("M=%d box=%s: D=%.15e exact=%.15e gap=%.2e bound=%.2e"
          % (M, box, D, Dx, abs(D - Dx), bound))
    assert abs(D - Dx) <= 1.01 * bound + 1e-15 * abs(Dx)
    # the bound is tight enough to see a planted factor: well below |Dx|
    assert bound < 1e-2 * abs(Dx)


def test_diag_constant_equals_pair_sum_difference(soe_tables):
    """q_i D equals the difference of the direct pair sums (O2) with and without
    the j = i pair over the whole lattice (k = 0 and self terms left out)."""
    w, s = soe_tables[16]
    box = (9.0, 7.0, 3.0)
    alpha = 0.8
    pos, q = wl.random_system(6, box, seed=31)
    q = q * np.array([1.0, 2.0, 1.0, 0.5, 1.0, 1.5])
    modes, wts = soewald2d.exact_modes(box[0], box[1], alpha, 2 * alpha * np.sqrt(np.log(1e18)))
    a = soewald2d.long_range(pos, q, box, alpha, w, s, modes, wts, include_self_pair=True, k0=False)
    b = soewald2d.long_range(pos, q, box, alpha, w, s, modes, wts, include_self_pair=False, k0=False)
    D = soewald2d.diag_constant(box[0], box[1], alpha, w, s)
    np.testing.assert_allclose(a["phi"] - b["phi"], q * D, rtol=1e-10, atol=1e-14)


def test_diag_constant_pin_catches_planted_mistakes(soe_tables, monkeypatch):
    """A factor 2 in D, or a wrong Gaussian (e^{-k^2/(4 alpha)}, the printed form
    of the garbled factor), planted in the oracle, fails the j = i pin."""
    w, s = soe_tables[16]
    Lx, Ly, alpha = 20.0, 20.0, 0.4
    Dx, k = _diag_exact(Lx, Ly, alpha)
    eps = _eps(w, s)
    g = np.exp(-k * k / (4 * alpha * alpha))
    bound = np.pi / (Lx * Ly) * float(np.sum(4 * alpha * g * eps / (np.sqrt(np.pi) * k * k)))
    D = soewald2d.diag_constant(Lx, Ly, alpha, w, s)
    assert abs(2 * D - Dx) > 100 * bound
    real_exp = np.exp

    def wrong_gauss(x, *a, **kw):
        return real_exp(x * alpha, *a, **kw) if np.ndim(x) == 0 and x < 0 else real_exp(x, *a, **kw)

    monkeypatch.setattr(soewald2d.np, "exp", wrong_gauss)
    Dw = soewald2d.diag_constant(Lx, Ly, alpha, w, s)
    monkeypatch.undo()
    assert abs(Dw - Dx) > 100 * bound
