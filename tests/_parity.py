"""Parity measures shared by the GPU tests.

rel: relative L2 error over all particles (the paper's relative RMS).
assert_close: that norm within tol AND a per-particle bound, so that a few
bad particles (one mis-indexed segment among thousands) cannot hide under
the norm: max_i |a_i - r_i| <= factor * tol * RMS_i |r_i|, with |.| the
Euclidean norm of particle i's row (force vectors) or its absolute value.
"""
import numpy as np

PER_PARTICLE_FACTOR = 10.0


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def per_particle(a, b):
    """max_i |a_i - b_i| / RMS_i |b_i|."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.size == 0:
        return 0.0
    d = a - b
    if d.ndim > 1:
        d = np.sqrt((d * d).sum(axis=-1))
        r = np.sqrt((b * b).sum(axis=-1))
    else:
        d = np.abs(d)
        r = np.abs(b)
    rms = np.sqrt(np.mean(r * r))
    return float(d.max() / max(rms, 1e-300))


def assert_close(a, b, tol, what=""):
    e = rel(a, b)
    m = per_particle(a, b)
    assert np.all(np.isfinite(np.asarray(a, dtype=np.float64))), (what, "non-finite")
    assert e < tol, (what, "relative L2", e, tol)
    assert m <= PER_PARTICLE_FACTOR * tol, (what, "per particle", m, PER_PARTICLE_FACTOR * tol)
    return e, m


def assert_energy(E, U, q, phi_ref, tol, what="E"):
    """|E - U| within tol of max(|U|, 1/2 ||q phi_ref||_2): rounding errors of
    the per-particle potentials enter E = 1/2 sum q_i phi_i as a random sum,
    whose size is set by the L2 norm of the terms, not by the (cancelling)
    total of a neutral system."""
    q = np.asarray(q, dtype=np.float64)
    scale = max(abs(U), 0.5 * float(np.linalg.norm(q * np.asarray(phi_ref, dtype=np.float64))))
    assert abs(E - U) <= tol * scale, (what, abs(E - U), tol * scale, abs(U))
    return abs(E - U) / max(abs(U), 1e-300)
