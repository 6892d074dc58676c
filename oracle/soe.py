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


def load_table(path):
    """Read a table written by tests/golden/gen_soe_tables.py.

    Format: one line per term, 'Re(w) Im(w) Re(s) Im(s)' in %.17e.
    """
    a = np.loadtxt(path, comments="#", ndmin=2)
    return a[:, 0] + 1j * a[:, 1], a[:, 2] + 1j * a[:, 3]
