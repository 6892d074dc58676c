"""Brute-force lattice sums (oracle pins).

* ``direct_energy`` / ``direct_forces``: the pairwise Coulomb lattice sum of
  Sec. 2.1 (eq. U_pair), truncated on the symmetric disc |m| <= R of image
  indices, which Thm 2.1 shows converges for a neutral cell.  The caller
  extrapolates R -> infinity (``extrapolate``).
* ``H_direct`` / ``H_poisson``: the importance-sampling normaliser of Sec. 4.1,
  H = sum_{k != 0} exp(-k^2/(4 alpha^2)), by direct summation and by its
  Poisson-summation closed form.  Reading of a garbled formula: the printed
  closed form has alpha where Poisson summation of a Gaussian gives alpha^2;
  the form used is (alpha^2 Lx Ly / pi) sum_n exp(-alpha^2 (nx^2 Lx^2 + ny^2 Ly^2)) - 1.

These are definitions, not approximations; they pin O1 and the H of the GPU
plan.
"""

import numpy as np


def _disc(R):
    r = int(np.ceil(R))
    mx, my = np.meshgrid(np.arange(-r, r + 1), np.arange(-r, r + 1), indexing="ij")
    keep = mx * mx + my * my <= R * R
    return mx[keep].astype(np.float64), my[keep].astype(np.float64)


def direct_energy(pos, q, box, R):
    """1/2 sum_{|m|<=R} sum_i sum'_j q_i q_j / |r_i - r_j + M|."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    Lx, Ly, _ = box
    mx, my = _disc(R)
    U = 0.0
    n = len(q)
    for i in range(n):
        for j in range(n):
            d = pos[i] - pos[j]
            x = d[0] + mx * Lx
            y = d[1] + my * Ly
            r = np.sqrt(x * x + y * y + d[2] * d[2])
            if i == j:
                r = r[(mx != 0) | (my != 0)]
            U += 0.5 * q[i] * q[j] * np.sum(1.0 / r)
    return U


def direct_forces(pos, q, box, R):
    """F_i = q_i sum_{|m|<=R} sum'_j q_j (r_i - r_j + M)/|r_i - r_j + M|^3."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    Lx, Ly, _ = box
    mx, my = _disc(R)
    n = len(q)
    F = np.zeros((n, 3))
    for i in range(n):
        for j in range(n):
            d = pos[i] - pos[j]
            x = d[0] + mx * Lx
            y = d[1] + my * Ly
            z = np.full_like(x, d[2])
            r2 = x * x + y * y + z * z
            keep = r2 > 0
            inv3 = np.where(keep, 1.0 / np.where(keep, r2, 1.0) ** 1.5, 0.0)
            F[i] += q[i] * q[j] * np.array([np.sum(x * inv3), np.sum(y * inv3), np.sum(z * inv3)])
    return F


def extrapolate(Rs, vals, order=3):
    """Least-squares fit v(R) = v_inf + sum_p c_p R^-p, p = 1..order; return v_inf."""
    Rs = np.asarray(Rs, dtype=np.float64)
    A = np.stack([np.ones_like(Rs)] + [Rs ** (-p) for p in range(1, order + 1)], axis=1)
    coef, *_ = np.linalg.lstsq(A, np.asarray(vals, dtype=np.float64), rcond=None)
    return coef[0]


def H_direct(Lx, Ly, alpha, tol=1e-18):
    """sum over k != 0 of exp(-k^2/(4 alpha^2)) by direct summation."""
    # exp(-k^2/4a^2) < tol  <=>  k > 2a sqrt(-ln tol)
    kmax = 2 * alpha * np.sqrt(-np.log(tol))
    mx_max = int(np.ceil(kmax * Lx / (2 * np.pi)))
    my_max = int(np.ceil(kmax * Ly / (2 * np.pi)))
    mx = np.arange(-mx_max, mx_max + 1)
    my = np.arange(-my_max, my_max + 1)
    gx = np.exp(-(2 * np.pi * mx / Lx) ** 2 / (4 * alpha * alpha))
    gy = np.exp(-(2 * np.pi * my / Ly) ** 2 / (4 * alpha * alpha))
    return float(np.sum(gx) * np.sum(gy) - 1.0)


def H_poisson(Lx, Ly, alpha, nmax=4):
    """Poisson-summation closed form of H (alpha^2 reading)."""
    n = np.arange(-nmax, nmax + 1)
    sx = np.sum(np.exp(-(alpha * n * Lx) ** 2))
    sy = np.sum(np.exp(-(alpha * n * Ly) ** 2))
    return float(alpha * alpha * Lx * Ly / np.pi * sx * sy - 1.0)
