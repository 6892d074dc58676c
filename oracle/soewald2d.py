"""O2: the SOE-approximated Ewald2D long-range sum as plain direct pair sums.

This is the definition the fast method reproduces exactly up to rounding
order (the recursion of Sec. 3.2 is an exact rearrangement of these sums).

Kernels (SOE table w_l, s_l with e^{-x^2} ~ sum_l w_l e^{-s_l |x|}, beta_l = alpha s_l):

* mode k != 0, pair kernel of eq. SOEphi without its Gaussian factor:
    K_k(z) = (2 alpha / (sqrt(pi) k)) sum_l w_l (2 beta_l e^{-k z} - 2 k e^{-beta_l z}) / (beta_l^2 - k^2)
  and its z derivative (eq. z-der, App. E):
    K'_k(z) = (2 alpha / sqrt(pi)) sum_l w_l (2 beta_l e^{-beta_l z} - 2 beta_l e^{-k z}) / (beta_l^2 - k^2).
  With the Gaussian, e^{-k^2/(4 alpha^2)} K_k(z) = (xi_M^+ + xi_M^-)(k, z) / k.
* mode k = 0 (eq. 32 and eq. dzphi_0):
    K_0(z)  = sum_l (w_l/sqrt(pi)) [2z/s_l + (1/alpha - 2z/s_l) e^{-beta_l z}]
    K'_0(z) = sum_l (w_l/sqrt(pi)) [2/s_l - (s_l + 2/s_l - 2 alpha z) e^{-beta_l z}].

Potential on particle i (long-range part, the quantity q2d_long_range returns):
  phi_i = sum_modes omega_k sum_j q_j cos(k.rho_ij) K_k(|z_ij|)
          - (2 pi/A) sum_j q_j K_0(|z_ij|) - 2 alpha q_i / sqrt(pi)
with the j = i term included (Sec. 2.2 convention: phi_l includes the
Gaussian cloud's action on its own charge, phi_self removes it).  The sum over
k runs over the full lattice (k and -k), so only the real part cos(k.rho)
remains.  Forces F_i = -grad_i of the pair energy:
  F_rho,i = q_i sum_modes omega_k k_vec sum_{j!=i} q_j sin(k.rho_ij) K_k(|z_ij|)
  F_z,i   = -q_i sum_modes omega_k sum_{j!=i} q_j cos(k.rho_ij) sgn(z_i-z_j) K'_k(|z_ij|)
            + (2 pi/A) q_i sum_{j!=i} q_j sgn(z_i-z_j) K'_0(|z_ij|).
Energy U = 1/2 sum_i q_i phi_i.

Mode sets and weights:
* exact-k (Alg. 1): all 0 < |k| <= k_c, omega_k = (pi/A) e^{-k^2/(4 alpha^2)}.
* random batch (Sec. 4.1, eq. RBapp): a list of P sampled modes k_eta, each
  with omega = (pi/A) H / P (the Gaussian of the mode cancels against the
  sampling density h(k) = e^{-k^2/4alpha^2}/H).  The estimator covers the
  pairs j != i; the configuration-independent j = i constant, which the
  paper's phi-tilde drops, is added deterministically as q_i * D with
  D = (pi/A) sum_{k != 0} e^{-k^2/(4 alpha^2)} K_k(0) over the whole lattice
  (a reading: it keeps the estimator's energy on the same convention as the
  exact-k sum without adding variance).  A sampled mode enters as the real
  part of its complex pair sum, which is the average of k and -k and keeps
  the estimator unbiased because h(k) = h(-k).

Ties z_i = z_j (j != i) take sgn = 0 here.

Pins (tests/test_oracle_soewald2d.py): |K_k e^{-k^2/4a^2} - (xi^+ + xi^-)/k| and
the k=0 kernels against the exact kernels within the SOE error bounds of
Thm 3.2 and eq. erfSOE; O2 -> O1 as M grows; F = -grad U by central
differences; K'_k(0) = 0.
"""

import numpy as np

SQRT_PI = np.sqrt(np.pi)


def mode_k(mx, my, Lx, Ly):
    kx = 2 * np.pi * np.asarray(mx, dtype=np.float64) / Lx
    ky = 2 * np.pi * np.asarray(my, dtype=np.float64) / Ly
    return kx, ky, np.hypot(kx, ky)


def kernel_k(k, z, alpha, w, s):
    """(K_k(z), K'_k(z)) for scalar k > 0 and array z >= 0 (real parts)."""
    z = np.abs(np.asarray(z, dtype=np.float64))
    beta = alpha * s
    den = beta * beta - k * k
    ek = np.exp(-k * z)
    K = np.zeros(z.shape, dtype=np.complex128)
    Kd = np.zeros(z.shape, dtype=np.complex128)
    for wl, bl, dl in zip(w, beta, den):
        el = np.exp(-bl * z)
        K += wl * (2 * bl * ek - 2 * k * el) / dl
        Kd += wl * (2 * bl * el - 2 * bl * ek) / dl
    return (2 * alpha / (SQRT_PI * k) * K).real, (2 * alpha / SQRT_PI * Kd).real


def kernel_0(z, alpha, w, s):
    """(K_0(z), K'_0(z)) for array z >= 0 (eq. 32, eq. dzphi_0)."""
    z = np.abs(np.asarray(z, dtype=np.float64))
    K = np.zeros(z.shape, dtype=np.complex128)
    Kd = np.zeros(z.shape, dtype=np.complex128)
    for wl, sl in zip(w, s):
        el = np.exp(-alpha * sl * z)
        K += wl / SQRT_PI * (2 * z / sl + (1 / alpha - 2 * z / sl) * el)
        Kd += wl / SQRT_PI * (2 / sl - (sl + 2 / sl - 2 * alpha * z) * el)
    return K.real, Kd.real


def exact_modes(Lx, Ly, alpha, kc):
    """Full-lattice modes 0 < |k| <= kc and weights (pi/A) e^{-k^2/4a^2}."""
    from .ewald2d import kmodes_full
    m = kmodes_full(Lx, Ly, kc)
    _, _, k = mode_k(m[:, 0], m[:, 1], Lx, Ly)
    return m, np.pi / (Lx * Ly) * np.exp(-k * k / (4 * alpha * alpha))


def rb_weights(P, H, Lx, Ly):
    return np.full(P, np.pi / (Lx * Ly) * H / P)


def diag_constant(Lx, Ly, alpha, w, s, kc=None, tol=1e-18):
    """D = (pi/A) sum_{0<|k|(<=kc)} e^{-k^2/4a^2} K_k(0), summed directly."""
    if kc is None:
        kc = 2 * alpha * np.sqrt(-np.log(tol))
    from .ewald2d import kmodes_full
    m = kmodes_full(Lx, Ly, kc)
    _, _, k = mode_k(m[:, 0], m[:, 1], Lx, Ly)
    tot = 0.0
    for kk in k:
        K0, _ = kernel_k(kk, np.zeros(1), alpha, w, s)
        tot += np.exp(-kk * kk / (4 * alpha * alpha)) * K0[0]
    return np.pi / (Lx * Ly) * tot


def long_range(pos, q, box, alpha, w, s, modes, weights, targets=None,
               include_self_pair=True, diag=0.0, chunk=1 << 15, k0=True):
    """phi, F, (and U when targets is None) by direct pair sums.

    modes: (n, 2) integer (mx, my); weights: (n,) omega per mode.
    include_self_pair: add the j = i term of the k != 0 modes (exact-k);
    diag: constant D added as q_i * D (random-batch convention).
    targets: indices of particles to evaluate (default all).
    k0: include the k = 0 term and the self term (False leaves only the
    k != 0 modes and the diagonal constant).
    """
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    w = np.asarray(w, dtype=np.complex128)
    s = np.asarray(s, dtype=np.complex128)
    Lx, Ly, _ = box
    A = Lx * Ly
    N = len(q)
    modes = np.asarray(modes, dtype=np.int64).reshape(-1, 2)
    weights = np.asarray(weights, dtype=np.float64)
    kx, ky, kk = mode_k(modes[:, 0], modes[:, 1], Lx, Ly)
    beta = alpha * s
    # per-mode, per-term coefficients of the two exponentials in K_k and K'_k
    den = beta[None, :] ** 2 - kk[:, None] ** 2                      # (n, M)
    c_k = 2 * alpha / (SQRT_PI * kk[:, None]) * w[None, :] / den     # (n, M)
    c_d = 2 * alpha / SQRT_PI * w[None, :] / den                     # (n, M)
    ak = (c_k * 2 * beta[None, :]).sum(1).real                      # coef of e^{-kz} in K
    akd = -(c_d * 2 * beta[None, :]).sum(1).real                    # coef of e^{-kz} in K'
    al = -c_k * 2 * kk[:, None]                                     # coef of e^{-beta z} in K
    ald = c_d * 2 * beta[None, :]                                   # coef of e^{-beta z} in K'
    tg = np.arange(N) if targets is None else np.asarray(targets, dtype=np.int64)
    phi = np.zeros(len(tg))
    F = np.zeros((len(tg), 3))
    for t, i in enumerate(tg):
        acc_phi = 0.0
        acc_f = np.zeros(3)
        for j0 in range(0, N, chunk):
            j1 = min(N, j0 + chunk)
            dx = pos[i, 0] - pos[j0:j1, 0]
            dy = pos[i, 1] - pos[j0:j1, 1]
            dz = pos[i, 2] - pos[j0:j1, 2]
            az = np.abs(dz)
            sg = np.sign(dz)
            qj = q[j0:j1]
            self_mask = (np.arange(j0, j1) == i)
            E = np.exp(-np.outer(beta, az))                                   # (M, n)
            Ek = np.exp(-np.outer(kk, az))                                    # (modes, n)
            K = ak[:, None] * Ek + (al @ E).real                              # (modes, n)
            Kd = akd[:, None] * Ek + (ald @ E).real
            th = np.outer(kx, dx) + np.outer(ky, dy)
            c = np.cos(th)
            sn = np.sin(th)
            qpair = np.where(self_mask, 0.0, qj)
            qphi = qj if include_self_pair else qpair
            acc_phi += float(weights @ ((c * K) @ qphi))
            fr = weights * ((sn * K) @ qpair)
            acc_f[0] += q[i] * float(kx @ fr)
            acc_f[1] += q[i] * float(ky @ fr)
            acc_f[2] += -q[i] * float(weights @ ((c * Kd) @ (qpair * sg)))
            if k0:
                # k = 0 term, j = i included in phi
                K0, K0d = kernel_0(az, alpha, w, s)
                acc_phi += -(2 * np.pi / A) * float(K0 @ qj)
                acc_f[2] += (2 * np.pi / A) * q[i] * float(K0d @ (qpair * sg))
        phi[t] = acc_phi + q[i] * diag - (2 * alpha * q[i] / SQRT_PI if k0 else 0.0)
        F[t] = acc_f
    out = dict(phi=phi, F=F)
    if targets is None:
        out["U"] = 0.5 * float(q @ phi)
    return out


def exact_k(pos, q, box, alpha, kc, w, s, targets=None):
    """SOEwald2D long-range part over all 0 < |k| <= kc (Alg. 1)."""
    m, wt = exact_modes(box[0], box[1], alpha, kc)
    return long_range(pos, q, box, alpha, w, s, m, wt, targets=targets)


def rb(pos, q, box, alpha, w, s, modes, H, targets=None, diag=None):
    """Random-batch estimator for a given list of sampled modes (eq. RBapp)."""
    modes = np.asarray(modes).reshape(-1, 2)
    if diag is None:
        diag = diag_constant(box[0], box[1], alpha, w, s)
    return long_range(pos, q, box, alpha, w, s, modes,
                      rb_weights(len(modes), H, box[0], box[1]),
                      targets=targets, include_self_pair=False, diag=diag)
