"""Pins of the particle-slab oracle (Sec. 2.4) and of the Langevin step (Sec. 4.3)."""
import numpy as np

import workloads as wl
from oracle import ewald2d, slabs


def _probes(box, zs, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(zs)
    return np.stack([rng.uniform(0, box[0], n), rng.uniform(0, box[1], n), np.asarray(zs)], 1)


def test_zero_mode_is_the_uniform_closed_form():
    """Thm 2.7 with only the zero mode (uniform walls, sig(0) = sigma A) equals
    eq. spectial on [0, Lz], and the potential is linear in z there."""
    box = (7.0, 5.0, 3.0)
    A = box[0] * box[1]
    pos, q = wl.random_system(40, box, seed=3)
    sb, st = 0.31, -0.17
    u = slabs.slab_uniform(pos, q, box, sb, st)
    g = slabs.slab_series(pos, q, box, np.zeros((0, 2), int), [], [], sb * A, st * A)
    np.testing.assert_allclose(g["phi"], u["phi"], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(g["F"], u["F"], rtol=1e-13, atol=1e-13)
    z = np.linspace(0, box[2], 7)
    p = slabs.slab_uniform(np.stack([np.zeros(7), np.zeros(7), z], 1), np.ones(7), box, sb, st)
    assert np.abs(np.diff(p["phi"], 2)).max() < 1e-12  # linear in z
    # the field of two sheets: F_z = 2 pi q (sigma_bot - sigma_top) between them
    np.testing.assert_allclose(u["F"][:, 2], 2 * np.pi * q * (sb - st), rtol=1e-14)


def test_series_against_point_charge_wall_with_exact_ewald():
    """Walls with sinusoidal densities, discretised into a fine grid of point
    charges, evaluated with the exact Ewald2D oracle (O1) at probe points away
    from the walls: equal to the Thm 2.7 series up to the grid's aliasing error
    (about e^{-2 pi G z / L})."""
    box = (10.0, 8.0, 4.0)
    Lx, Ly, Lz = box
    A = Lx * Ly
    G = 48
    xa = (np.arange(G) + 0.5) * Lx / G
    ya = (np.arange(G) + 0.5) * Ly / G
    X, Y = np.meshgrid(xa, ya, indexing="ij")
    s0b, s1b, s0t, s2t = 0.05, 0.3, -0.12, 0.2
    sig_b = s0b + s1b * np.cos(2 * np.pi * X / Lx)
    sig_t = s0t + s2t * np.sin(2 * np.pi * (X / Lx + 2 * Y / Ly))
    dA = A / G ** 2
    wall = np.concatenate([np.stack([X.ravel(), Y.ravel(), np.zeros(G * G)], 1),
                           np.stack([X.ravel(), Y.ravel(), np.full(G * G, Lz)], 1)])
    qw = np.concatenate([sig_b.ravel(), sig_t.ravel()]) * dA
    probes = _probes(box, [1.0, 1.7, 2.2, 3.0, 1.3])
    pos = np.concatenate([wall, probes])
    q = np.concatenate([qw, np.zeros(len(probes))])
    tg = np.arange(len(wall), len(pos))
    alpha, s = 1.2, 5.0
    rc, kc = s / alpha, 2 * s * alpha
    ps, _ = ewald2d.real_space(pos, q, box, alpha, rc, targets=tg)
    pk, _ = ewald2d.fourier_k(pos, q, box, alpha, kc, targets=tg)
    p0, _ = ewald2d.fourier_0(pos, q, box, alpha, targets=tg)
    phi_pc = ps + pk + p0
    # Fourier coefficients over one cell: cos(2 pi x/Lx) -> modes (+-1, 0) with
    # A/2 each; sin(2 pi (x/Lx + 2y/Ly)) -> (1, 2): A/(2i), (-1, -2): -A/(2i)
    modes = np.array([[1, 0], [-1, 0], [1, 2], [-1, -2]])
    cb = np.array([s1b * A / 2, s1b * A / 2, 0, 0], dtype=complex)
    ct = np.array([0, 0, s2t * A / 2j, -s2t * A / 2j], dtype=complex)
    r = slabs.slab_series(probes, np.ones(len(probes)), box, modes, cb, ct, s0b * A, s0t * A)
    err = np.abs(phi_pc - r["phi"]).max()
    print("wall series vs point-charge Ewald2D: max |dphi| = %.2e (|phi| ~ %.2e)"
          % (err, np.abs(r["phi"]).max()))
    assert err < 1e-6 * max(1.0, np.abs(r["phi"]).max())


def test_series_force_is_minus_gradient():
    box = (6.0, 9.0, 5.0)
    A = box[0] * box[1]
    modes = np.array([[1, 1], [-1, -1], [0, 2], [0, -2], [3, -1], [-3, 1]])
    cb = np.array([0.4 + 0.2j, 0.4 - 0.2j, -0.3j, 0.3j, 0.05, 0.05])
    ct = np.array([0.1, 0.1, 0.25 + 0.1j, 0.25 - 0.1j, -0.02j, 0.02j])
    pos = _probes(box, [0.4, 2.5, 4.6, 3.3], seed=4)
    q = np.array([1.0, -2.0, 0.5, 1.5])
    r = slabs.slab_series(pos, q, box, modes, cb, ct, 0.2 * A, -0.1 * A)
    h = 1e-6
    for i in range(len(q)):
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, c] += h
            pm[i, c] -= h
            fp = slabs.slab_series(pp, q, box, modes, cb, ct, 0.2 * A, -0.1 * A)["phi"][i]
            fm = slabs.slab_series(pm, q, box, modes, cb, ct, 0.2 * A, -0.1 * A)["phi"][i]
            assert abs(-q[i] * (fp - fm) / (2 * h) - r["F"][i, c]) < 1e-7


def _harmonic_run(n, steps, dt, gamma, kT, kappa, seed, box=(1e3, 1e3, 1e3)):
    """BAOAB on n independent particles in the potential kappa/2 |r - c|^2."""
    c = np.array(box) / 2
    pos = np.tile(c, (n, 1)) + 0.1
    mom = np.zeros((n, 3))
    mass = np.full(n, 1.3)
    F = -kappa * (pos - c)
    xs = []
    for t in range(steps):
        pos, mom = slabs.baoab_first(pos, mom, mass, F, box, dt, gamma, kT, seed, t)
        F = -kappa * (pos - c)
        mom = slabs.baoab_second(mom, F, dt)
        xs.append(pos - c)
    return np.array(xs), mom, mass


def test_baoab_without_friction_is_velocity_verlet():
    """gamma = 0: the splitting is velocity Verlet; a harmonic oscillator's
    energy error is second order in dt and bounded (symplectic)."""
    errs = []
    for dt in (0.02, 0.01):
        xs, mom, mass = _harmonic_run(1, int(20 / dt), dt, 0.0, 1.0, 2.0, 0)
        E0 = 0.5 * 2.0 * 3 * 0.1 ** 2
        E = 0.5 * 2.0 * (xs[-1] ** 2).sum() + (mom ** 2).sum() / (2 * mass[0])
        errs.append(abs(E - E0))
    assert errs[0] < 1e-3 and 3.0 < errs[0] / errs[1] < 5.0


def test_baoab_samples_harmonic_configurations_exactly():
    """BAOAB samples <x^2> = kT / kappa of a harmonic oscillator exactly at any
    stable dt (Leimkuhler-Matthews); momenta relax to <p^2/m> = kT."""
    kT, kappa, dt = 0.7, 3.0, 0.35
    xs, mom, mass = _harmonic_run(4000, 400, dt, 2.0, kT, kappa, 11)
    x2 = (xs[200:] ** 2).mean()
    assert abs(x2 - kT / kappa) < 0.02 * kT / kappa
    p2 = (mom ** 2 / mass[:, None]).mean()
    assert abs(p2 - kT) < 0.1 * kT


def test_walls_reflect_and_wrap():
    box = (5.0, 4.0, 2.0)
    pos = np.array([[4.9, 0.1, 0.05], [0.1, 3.9, 1.95], [2.0, 2.0, 1.0]])
    mom = np.array([[1.0, -1.0, -2.0], [-1.0, 1.0, 3.0], [0.0, 0.0, 0.0]])
    F = np.zeros((3, 3))
    p2, m2 = slabs.baoab_first(pos, mom, np.ones(3), F, box, 0.1, 0.0, 1.0, 1, 0)
    assert np.all((p2[:, 0] >= 0) & (p2[:, 0] < box[0]) & (p2[:, 1] >= 0) & (p2[:, 1] < box[1]))
    assert np.all((p2[:, 2] >= 0) & (p2[:, 2] <= box[2]))
    np.testing.assert_allclose(p2[0], [0.0, 0.0, 0.15], atol=1e-12)
    assert m2[0, 2] == 2.0 and m2[1, 2] == -3.0
    np.testing.assert_allclose(p2[1, 2], 2 * 2.0 - (1.95 + 0.3), atol=1e-12)
