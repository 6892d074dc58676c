"""O1: the exact Ewald2D sum, FP64, plain O(N^2) loops (oracle).

Follows Sec. 2.2 of the paper:
  phi(r_i) = phi_s(r_i) + phi_l(r_i) - phi_self^i                (Ewald split)
  phi_s   = sum_m sum'_j q_j erfc(alpha|r_ij+M|)/|r_ij+M|          (real space)
  phi_self = 2 alpha q_i / sqrt(pi)                                (self term)
  phi_l   = sum_{k != 0} phi^k + phi^0                             (Lemma 2.4)
  phi^k(r_i) = (pi/A) sum_j q_j e^{i k.rho_ij}/k [xi^+ + xi^-](k, |z_ij|),
  xi^{+-}(k,z) = e^{+-kz} erfc(k/(2 alpha) +- alpha z),
  phi^0(r_i) = -(2 pi/A) sum_j q_j [z_ij erf(alpha z_ij) + e^{-alpha^2 z_ij^2}/(alpha sqrt(pi))].
The j = i term is part of phi_l (the Gaussian cloud acting on its own point
charge); phi_self removes it again in the limit.  Energy U = 1/2 sum q_i phi_i
(pair energy of Sec. 2.1), force F_i = -grad_i U.

The Fourier sum runs over the full lattice 0 < |k| <= k_c (both k and -k).
xi^{+-} are evaluated without overflow through erfcx:
  xi^+ = erfcx(u+) e^{-k^2/4a^2 - a^2 z^2},  u+ = k/2a + a z
  xi^- = erfcx(u-) e^{-k^2/4a^2 - a^2 z^2}                      (u- >= 0)
       = 2 e^{-kz} - erfcx(-u-) e^{-k^2/4a^2 - a^2 z^2}         (u- < 0)
and d/dz [xi^+ + xi^-] = k (xi^+ - xi^-).  The k = 0 force uses
d/dz [z erf(a z) + e^{-a^2 z^2}/(a sqrt(pi))] = erf(a z).

Pins (tests/test_oracle_ewald2d.py): the Madelung constant of the square
2-D ionic lattice (all ions in one plane), brute-force direct lattice sums of
Sec. 2.1 on 2-4 charges (Thm 2.1 summation shape), independence of U and F
from alpha, and F = -grad U by central differences.
"""

import numpy as np
from scipy.special import erfc, erf, erfcx

SQRT_PI = np.sqrt(np.pi)


def _check(pos, q):
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if pos.ndim != 2 or pos.shape[1] != 3 or q.shape != (pos.shape[0],):
        raise ValueError("pos must be N x 3 and q of length N")
    return pos, q


def kmodes_full(Lx, Ly, kc):
    """All (mx, my) != 0 with |k| <= kc, k = 2 pi (mx/Lx, my/Ly)."""
    mx_max = int(np.floor(kc * Lx / (2 * np.pi)))
    my_max = int(np.floor(kc * Ly / (2 * np.pi)))
    out = []
    for mx in range(-mx_max, mx_max + 1):
        for my in range(-my_max, my_max + 1):
            if mx == 0 and my == 0:
                continue
            kx, ky = 2 * np.pi * mx / Lx, 2 * np.pi * my / Ly
            if kx * kx + ky * ky <= kc * kc:
                out.append((mx, my))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def xi_sum(k, z, alpha):
    """(xi^+ + xi^-, xi^+ - xi^-) at z >= 0 (Lemma 2.4), overflow-free."""
    z = np.abs(z)
    g = np.exp(-k * k / (4 * alpha * alpha) - alpha * alpha * z * z)
    up = k / (2 * alpha) + alpha * z
    um = k / (2 * alpha) - alpha * z
    xp = erfcx(up) * g
    xm = np.where(um >= 0, erfcx(np.abs(um)) * g, 2 * np.exp(-k * z) - erfcx(np.abs(um)) * g)
    return xp + xm, xp - xm


def real_space(pos, q, box, alpha, rc, targets=None):
    """phi_s and F_s (eq. phi_s): truncated erfc sum over images within rc.
    targets: indices of the particles to evaluate (default all); every
    particle is a source either way."""
    pos, q = _check(pos, q)
    Lx, Ly, _ = box
    tg = np.arange(len(q)) if targets is None else np.asarray(targets, dtype=np.int64)
    n = len(tg)
    phi = np.zeros(n)
    F = np.zeros((n, 3))
    nx = int(np.ceil(rc / Lx)) + 1
    ny = int(np.ceil(rc / Ly)) + 1
    d0 = pos[tg, None, :] - pos[None, :, :]
    same = tg[:, None] == np.arange(len(q))[None, :]
    for mx in range(-nx, nx + 1):
        for my in range(-ny, ny + 1):
            d = d0 + np.array([mx * Lx, my * Ly, 0.0])
            r = np.sqrt((d * d).sum(-1))
            mask = r <= rc
            if mx == 0 and my == 0:
                mask &= ~same
            if not mask.any():
                continue
            rs = np.where(mask, r, 1.0)
            e = np.where(mask, erfc(alpha * rs) / rs, 0.0)
            phi += e @ q
            fm = np.where(mask, (erfc(alpha * rs) / rs ** 2
                                 + 2 * alpha / SQRT_PI * np.exp(-(alpha * rs) ** 2) / rs) / rs, 0.0)
            F += q[tg, None] * ((fm * q[None, :])[:, :, None] * d).sum(1)
    return phi, F


def fourier_k(pos, q, box, alpha, kc, targets=None):
    """sum over 0 < |k| <= kc of phi^k and its force (eq. philk), full lattice.
    targets: indices of the particles to evaluate (default all)."""
    pos, q = _check(pos, q)
    Lx, Ly, _ = box
    A = Lx * Ly
    tg = np.arange(len(q)) if targets is None else np.asarray(targets, dtype=np.int64)
    n = len(tg)
    phi = np.zeros(n)
    F = np.zeros((n, 3))
    dx = pos[tg, None, 0] - pos[None, :, 0]
    dy = pos[tg, None, 1] - pos[None, :, 1]
    dz = pos[tg, None, 2] - pos[None, :, 2]
    az = np.abs(dz)
    sg = np.sign(dz)
    for mx, my in kmodes_full(Lx, Ly, kc):
        kx, ky = 2 * np.pi * mx / Lx, 2 * np.pi * my / Ly
        k = np.hypot(kx, ky)
        th = kx * dx + ky * dy
        G, Gd = xi_sum(k, az, alpha)
        c = np.cos(th)
        s = np.sin(th)
        phi += (np.pi / A) * ((c * G / k) @ q)
        # -d/drho_i cos(k.rho_ij) = k sin(k.rho_ij)
        fr = (np.pi / A) * q[tg] * ((s * G / k) @ q)
        F[:, 0] += kx * fr
        F[:, 1] += ky * fr
        # d/dz_i G(|z_ij|) = sgn(z_ij) k (xi+ - xi-)
        F[:, 2] += -(np.pi / A) * q[tg] * ((c * sg * Gd) @ q)
    return phi, F


def fourier_0(pos, q, box, alpha, targets=None):
    """phi^0 and its z force (eq. phil0); targets as in fourier_k."""
    pos, q = _check(pos, q)
    Lx, Ly, _ = box
    A = Lx * Ly
    tg = np.arange(len(q)) if targets is None else np.asarray(targets, dtype=np.int64)
    dz = pos[tg, None, 2] - pos[None, :, 2]
    az = np.abs(dz)
    K = az * erf(alpha * az) + np.exp(-(alpha * az) ** 2) / (alpha * SQRT_PI)
    phi = -(2 * np.pi / A) * (K @ q)
    F = np.zeros((len(tg), 3))
    F[:, 2] = (2 * np.pi / A) * q[tg] * ((np.sign(dz) * erf(alpha * az)) @ q)
    return phi, F


def self_term(q, alpha):
    """phi_self^i = 2 alpha q_i / sqrt(pi) (eq. self)."""
    return 2 * alpha * np.asarray(q, dtype=np.float64) / SQRT_PI


def ewald2d(pos, q, box, alpha, rc, kc):
    """Full Ewald2D: returns dict(phi, F, U) and the parts."""
    pos, q = _check(pos, q)
    ps, Fs = real_space(pos, q, box, alpha, rc)
    pk, Fk = fourier_k(pos, q, box, alpha, kc)
    p0, F0 = fourier_0(pos, q, box, alpha)
    pself = self_term(q, alpha)
    phi = ps + pk + p0 - pself
    F = Fs + Fk + F0
    return dict(phi=phi, F=F, U=0.5 * float(q @ phi), phi_s=ps, F_s=Fs,
                phi_k=pk, F_k=Fk, phi_0=p0, F_0=F0, phi_self=pself)


def long_range(pos, q, box, alpha, kc):
    """phi_l - phi_self and its force: the quantity the long-range solver returns."""
    pos, q = _check(pos, q)
    pk, Fk = fourier_k(pos, q, box, alpha, kc)
    p0, F0 = fourier_0(pos, q, box, alpha)
    phi = pk + p0 - self_term(q, alpha)
    return dict(phi=phi, F=Fk + F0, U=0.5 * float(q @ phi))
