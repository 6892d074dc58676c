"""Sum-of-exponentials (SOE) approximation of the Gaussian (oracle side).

The paper (Sec. 3, opening) writes an M-term SOE of a kernel f as
``|f(x) - sum_l w_l exp(-s_l |x|)| <= eps`` for all real x, and obtains the
Gaussian's SOE by discretising its inverse-Laplace (Bromwich) representation
along a contour.  The paper itself uses VPMR nodes, which it does not list;
this module builds its own table by the midpoint rule on Weideman's optimised
Talbot contour.

Reading of a garbled formula: the printed representation has exp(-sqrt(z)|x|);
the Laplace pair L^{-1}[exp(-a sqrt(p))/sqrt(p)](t=1) = exp(-a^2/4)/sqrt(pi)
fixes the exponent as exp(-2 sqrt(z)|x|), which is what is used here:

    exp(-x^2) = (1/2 pi i) int_Gamma e^z sqrt(pi/z) exp(-2 sqrt(z) |x|) dz.

With nodes z_k on the contour and step h, s_k = 2 sqrt(z_k) (principal root,
Re s_k > 0) and w_k = h/(2 pi i) e^{z_k} sqrt(pi/z_k) z'(theta_k).  An even
node count on a contour symmetric about the real axis gives complex-conjugate
pairs only.

Pins (tests/test_oracle_soe.py): the sup-norm error on a dense grid, the
moments sum(w) = 1 (value at 0) and sum(w/s) = sqrt(pi)/2 (integral over the
half line), and symmetry of the table under conjugation.
"""

import numpy as np

# Weideman (2006), "Optimizing Talbot's contours for the inversion of the
# Laplace transform": z(theta) = N (sigma + mu theta cot(a theta) + i nu theta).
_TALBOT_SIGMA = -0.6122
_TALBOT_MU = 0.5017
_TALBOT_A = 0.6407
_TALBOT_NU = 0.2645


def talbot_soe(M, scale=1.0):
    """Return (w, s), complex arrays of length M, for exp(-x^2).

    M must be even so that the nodes come in conjugate pairs.  ``scale``
    multiplies the contour size N = M (the classical choice is 1).
    """
    if M < 2 or M % 2:
        raise ValueError("M must be an even integer >= 2")
    h = 2.0 * np.pi / M
    th = -np.pi + (np.arange(M) + 0.5) * h
    n = M * scale
    a = _TALBOT_A
    z = n * (_TALBOT_SIGMA + _TALBOT_MU * th / np.tan(a * th) + 1j * _TALBOT_NU * th)
    dz = n * (_TALBOT_MU * (1.0 / np.tan(a * th) - a * th / np.sin(a * th) ** 2)
              + 1j * _TALBOT_NU)
    w = h / (2j * np.pi) * np.exp(z) * np.sqrt(np.pi / z) * dz
    s = 2.0 * np.sqrt(z)
    return w, s


def soe_eval(w, s, x):
    """sum_l w_l exp(-s_l |x|), real part (the table is conjugate-closed)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    return (np.exp(-np.multiply.outer(x, s)) @ w).real


def sup_error(w, s, xmax=200.0, n=400001):
    """Max |exp(-x^2) - SOE(x)| over a dense grid of [0, xmax]."""
    x = np.concatenate([np.linspace(0.0, 12.0, n), np.linspace(12.0, xmax, n // 10)])
    err = 0.0
    for chunk in np.array_split(x, 64):
        err = max(err, float(np.abs(soe_eval(w, s, chunk) - np.exp(-chunk ** 2)).max()))
    return err


def best_talbot_soe(M, scales=None):
    """Talbot table of size M with the contour scale that minimises sup error."""
    if scales is None:
        scales = np.linspace(0.6, 1.4, 41)
    best = None
    for sc in scales:
        w, s = talbot_soe(M, sc)
        e = sup_error(w, s, n=40001)
        if best is None or e < best[0]:
            best = (e, w, s)
    e, w, s = best
    return w, s, sup_error(w, s)


def _balanced_truncation_poles(w, s, M):
    """Exponents of the M-state balanced truncation of the SOE (w, s).

    The SOE sum_l w_l e^{-s_l x} is the impulse response C e^{A x} B of the
    linear system A = -diag(s), B_l = C_l = sqrt(w_l).  Its Gramians are
    Cauchy-like, P_ij = B_i conj(B_j) / (s_i + conj(s_j)) and
    Q_ij = conj(C_i) C_j / (conj(s_i) + s_j); with square roots P = Lp Lp^H,
    Q = Lq Lq^H and the SVD Lq^H Lp = U S V^H, the reduced system is
    A_r = S_r^{-1/2} U_r^H Lq^H A Lp V_r S_r^{-1/2}, whose eigenvalues are the
    new poles -s.  numpy's eigh, svd and eig serve as the steps."""
    B = np.sqrt(w + 0j)
    C = w / B
    P = np.outer(B, B.conj()) / (s[:, None] + s.conj()[None, :])
    Q = np.outer(C.conj(), C) / (s.conj()[:, None] + s[None, :])
    ep, vp = np.linalg.eigh(P)
    eq, vq = np.linalg.eigh(Q)
    Lp = vp * np.sqrt(np.clip(ep, 0, None))
    Lq = vq * np.sqrt(np.clip(eq, 0, None))
    U, S, Vh = np.linalg.svd(Lq.conj().T @ Lp)
    T = Lp @ Vh.conj().T[:, :M] / np.sqrt(S[:M])
    Ti = (U[:, :M].conj().T @ Lq.conj().T) / np.sqrt(S[:M])[:, None]
    Ar = Ti @ np.diag(-s) @ T
    return -np.linalg.eigvals(Ar)


def _pair_table(wp, sp):
    return np.concatenate([wp, wp.conj()]), np.concatenate([sp, sp.conj()])


def _fit_grid():
    return np.concatenate([np.linspace(0.0, 6.5, 3000), np.linspace(6.5, 40.0, 401)[1:]])


def _lsq_weights(sp, x):
    """Weights w_p of fixed pair exponents s_p (Im s_p > 0) minimising
    || 2 Re sum_p w_p e^{-s_p x} - e^{-x^2} || on the grid."""
    E = np.exp(-np.outer(x, sp))
    A = np.concatenate([2 * E.real, -2 * E.imag], axis=1)
    c, *_ = np.linalg.lstsq(A, np.exp(-x * x), rcond=None)
    h = len(sp)
    return c[:h] + 1j * c[h:]


def _lawson_lm(wp, sp, x, iters=1500):
    """Levenberg-Marquardt on (w_p, s_p) for the weighted residual, with the
    weights raised where the error is largest every 10 iterations (Lawson's
    route to the minimax fit); returns the iterate of smallest grid sup error."""
    h = len(wp)
    f = np.exp(-x * x)
    wt = np.ones_like(x)

    def value(w_, s_):
        return 2 * (np.exp(-np.outer(x, s_)) @ w_).real

    g = value(wp, sp)
    cost = np.sum((wt * (g - f)) ** 2)
    best = (np.abs(g - f).max(), wp.copy(), sp.copy())
    lam, since = 1e-3, 0
    for it in range(iters):
        E = np.exp(-np.outer(x, sp))
        xwE = x[:, None] * wp * E
        J = np.concatenate([2 * E.real, -2 * E.imag, -2 * xwE.real, 2 * xwE.imag], axis=1)
        J = J * wt[:, None]
        r = wt * (g - f)
        JtJ, Jtr = J.T @ J, J.T @ r
        stepped = False
        while lam < 1e10:
            d = np.linalg.solve(JtJ + lam * np.diag(np.diag(JtJ)), -Jtr)
            w2 = wp + d[:h] + 1j * d[h:2 * h]
            s2 = sp + d[2 * h:3 * h] + 1j * d[3 * h:]
            if np.all(s2.real > 0) and np.all(s2.imag > 0):
                g2 = value(w2, s2)
                c2 = np.sum((wt * (g2 - f)) ** 2)
                if c2 < cost:
                    wp, sp, g, cost = w2, s2, g2, c2
                    lam = max(lam / 3, 1e-12)
                    stepped = True
                    break
            lam *= 4
        if not stepped:
            break
        e = np.abs(g - f).max()
        since = 0 if e < best[0] * (1 - 1e-3) else since + 1
        if e < best[0]:
            best = (e, wp.copy(), sp.copy())
        if since > 300:
            break
        if it % 10 == 9:
            a = np.abs(g - f)
            wt = wt * np.sqrt(np.maximum(a / a.max(), 1e-3))
            wt /= wt.max()
            cost = np.sum((wt * (g - f)) ** 2)
    return best[1], best[2]


def reduced_soe(M, M_ref=48):
    """Model-reduced SOE of exp(-x^2) with M terms (M even, at most 12).

    The role of the paper's VPMR tables: balanced truncation of the M_ref-term
    Talbot table to M states (conjugate-pair poles), least-squares weights,
    then a Lawson-weighted Levenberg-Marquardt polish.  Returns (w, s, err)."""
    if M < 2 or M % 2 or M > 12:
        raise ValueError("M must be even, 2 <= M <= 12")
    w0, s0, _ = best_talbot_soe(M_ref)
    poles = _balanced_truncation_poles(w0, s0, M)
    sp = np.sort_complex(poles[poles.imag > 0])
    if len(sp) != M // 2:
        raise RuntimeError("reduced poles are not conjugate pairs")
    x = _fit_grid()
    wp = _lsq_weights(sp, x)
    wp, sp = _lawson_lm(wp, sp, x)
    w, s = _pair_table(wp, sp)
    return w, s, sup_error(w, s)


def load_table(path):
    """Read a table written by tests/golden/gen_soe_tables.py.

    Format: one line per term, 'Re(w) Im(w) Re(s) Im(s)' in %.17e.
    """
    a = np.loadtxt(path, comments="#", ndmin=2)
    return a[:, 0] + 1j * a[:, 1], a[:, 2] + 1j * a[:, 3]
