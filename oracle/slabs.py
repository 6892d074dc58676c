"""Particle-slab term and a Langevin integrator step (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Charged slabs (Sec. 2.4).  Two charged walls at z = 0 and z = Lz carry
doubly periodic surface charge densities sigma_bot(rho), sigma_top(rho).  The
particle-slab potential of Thm 2.7 (eq. phiionwall, eq. phionwallzero) is
  phi_ps(r) = (2 pi / A) sum_{k != 0} e^{i k.rho} / k
                 [sig_bot(k) e^{-k |z|} + sig_top(k) e^{-k |z - Lz|}]
              - (2 pi / A) [sig_bot(0) |z| + sig_top(0) |z - Lz|],
with sig(k) the 2-D Fourier coefficients of one cell.  Reading (the paper
refers to its lemma on 2-D Fourier transforms, which states the radial case
only): sig(k) = integral over [0, Lx) x [0, Ly) of sigma(rho) e^{-i k.rho},
so that sigma(rho) = (1/A) sum_k sig(k) e^{i k.rho} and sig(0) is the charge of
one cell of the wall; with this convention the zero mode reproduces the
uniform-slab closed form eq. spectial, phi_ps = -2 pi [sigma_top (Lz - z) +
sigma_bot z] on 0 <= z <= Lz.  The sum over k runs over a full lattice list
(k and -k both given), and the real part is taken (for real sigma the k and
-k terms are conjugate).  Forces F_i = -q_i grad phi_ps(r_i).  The
particle-slab energy is U_ps = sum_i q_i phi_ps(r_i) (reading: the walls are
external to the particles, so no factor 1/2; the wall-wall energy is a
configuration-independent constant and is left out).

Langevin step (Sec. 4.3, eq. langevin): dr = p/m dt, dp = (F - gamma p/m) dt +
sqrt(2 gamma / beta) dW.  The paper gives the SDE only; the discretisation
taken here is the BAOAB splitting (Leimkuhler and Matthews, 2013): a half
kick B, a half drift A, the exact Ornstein-Uhlenbeck step O
  p <- e^{-gamma dt/m} p + sqrt(m kT (1 - e^{-2 gamma dt/m})) xi,
a half drift, the force at the new positions, and a half kick.  Readings:
x, y wrap into [0, L) (periodic); the confining walls reflect specularly
(z -> -z, p_z -> -p_z below 0; z -> 2 Lz - z, p_z -> -p_z above Lz, repeated
if a step crosses both), applied once after the second half drift, which keeps
the Boltzmann distribution of a particle between the walls.  Normal
deviates: Philox4x32-10 (the generator of oracle/rbsampler.py) with key =
seed and counter (particle, step low, step high, stream), stream 3 giving
xi_x, xi_y and stream 4 giving xi_z, each pair by Box-Muller on two 53-bit
uniforms.

Pins (tests/test_oracle_slabs.py): the Thm 2.7 series with only the zero mode
equals eq. spectial and is linear in z between the walls; a sinusoidal wall
density against the potential of a point-charge discretisation of the wall
computed by the exact Ewald2D oracle (O1); BAOAB with gamma = 0 is
velocity Verlet (second-order energy error on a harmonic oscillator); BAOAB
samples a harmonic oscillator's <x^2> = kT / kappa exactly and free
momenta <p^2/m> = kT.
"""

import numpy as np

from .rbsampler import MASK, _u53, philox4x32_10_vec


def slab_uniform(pos, q, box, sigma_bot, sigma_top):
    """eq. spectial: phi_ps, F_ps, U_ps for uniform walls."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    Lz = box[2]
    z = pos[:, 2]
    phi = -2 * np.pi * (sigma_top * (Lz - z) + sigma_bot * z)
    F = np.zeros((len(q), 3))
    F[:, 2] = -q * (-2 * np.pi * (sigma_bot - sigma_top))
    return dict(phi=phi, F=F, U=float(q @ phi))


def slab_series(pos, q, box, modes, sig_bot, sig_top, sig0_bot, sig0_top):
    """Thm 2.7: phi_ps, F_ps, U_ps for walls with Fourier coefficients
    sig_bot[k], sig_top[k] on the full-lattice list `modes` ((n, 2) integers,
    no (0, 0)) and zero modes sig0_bot, sig0_top (charge per cell)."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    Lx, Ly, Lz = box
    A = Lx * Ly
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    modes = np.asarray(modes, dtype=np.int64).reshape(-1, 2)
    sig_bot = np.asarray(sig_bot, dtype=np.complex128)
    sig_top = np.asarray(sig_top, dtype=np.complex128)
    phi = np.zeros(len(q), dtype=np.complex128)
    gx = np.zeros(len(q), dtype=np.complex128)
    gy = np.zeros(len(q), dtype=np.complex128)
    gz = np.zeros(len(q), dtype=np.complex128)
    zb, zt = np.abs(z), np.abs(z - Lz)
    sb, st = np.sign(z), np.sign(z - Lz)
    for (mx, my), cb, ct in zip(modes, sig_bot, sig_top):
        kx, ky = 2 * np.pi * mx / Lx, 2 * np.pi * my / Ly
        k = np.hypot(kx, ky)
        ph = np.exp(1j * (kx * x + ky * y)) / k
        eb, et = np.exp(-k * zb), np.exp(-k * zt)
        term = (2 * np.pi / A) * ph * (cb * eb + ct * et)
        phi += term
        gx += 1j * kx * term
        gy += 1j * ky * term
        gz += (2 * np.pi / A) * ph * (-k) * (cb * sb * eb + ct * st * et)
    phi = phi.real - (2 * np.pi / A) * (sig0_bot * zb + sig0_top * zt)
    dz0 = -(2 * np.pi / A) * (sig0_bot * sb + sig0_top * st)
    F = np.stack([-q * gx.real, -q * gy.real, -q * (gz.real + dz0)], axis=1)
    return dict(phi=phi, F=F, U=float(q @ phi))


def normals(seed, step, n):
    """(n, 3) standard normal deviates of the Langevin step (see module text)."""
    k0, k1 = seed & MASK, (seed >> 32) & MASK
    idx = np.arange(n, dtype=np.uint64)
    out = np.zeros((n, 3))
    for col, stream in ((0, 3), (2, 4)):
        r0, r1, r2, r3 = philox4x32_10_vec(idx, step & MASK, (step >> 32) & MASK, stream, k0, k1)
        u1, u2 = _u53(r0, r1), _u53(r2, r3)
        rad = np.sqrt(-2.0 * np.log(u1))
        out[:, col] = rad * np.cos(2 * np.pi * u2)
        if col == 0:
            out[:, 1] = rad * np.sin(2 * np.pi * u2)
    return out


def _confine(pos, mom, box):
    """Wrap x, y; fold z into [0, Lz] by reflections at both walls (period
    2 Lz: an odd number of reflections, i.e. a folded height past Lz, flips p_z)."""
    Lx, Ly, Lz = box
    pos[:, 0] -= np.floor(pos[:, 0] / Lx) * Lx
    pos[:, 1] -= np.floor(pos[:, 1] / Ly) * Ly
    zf = pos[:, 2] - np.floor(pos[:, 2] / (2 * Lz)) * (2 * Lz)
    odd = zf > Lz
    pos[:, 2] = np.where(odd, 2 * Lz - zf, zf)
    mom[:, 2] = np.where(odd, -mom[:, 2], mom[:, 2])


def baoab_first(pos, mom, mass, F, box, dt, gamma, kT, seed, step):
    """B A O A of one step from forces F at the current positions: returns new
    (pos, mom); the caller computes forces at the new positions and finishes
    with baoab_second."""
    pos = np.array(pos, dtype=np.float64)
    mom = np.array(mom, dtype=np.float64)
    m = np.asarray(mass, dtype=np.float64).reshape(-1, 1) * np.ones((1, 3))
    mom += 0.5 * dt * np.asarray(F, dtype=np.float64)
    pos += 0.5 * dt * mom / m
    c1 = np.exp(-gamma * dt / m)
    mom = c1 * mom + np.sqrt(m * kT * (1.0 - c1 * c1)) * normals(seed, step, len(pos))
    pos += 0.5 * dt * mom / m
    _confine(pos, mom, box)
    return pos, mom


def baoab_second(mom, F, dt):
    """The closing half kick B with the forces at the new positions."""
    return np.asarray(mom, dtype=np.float64) + 0.5 * dt * np.asarray(F, dtype=np.float64)
