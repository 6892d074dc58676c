"""Random-batch mode sampler (oracle): Philox4x32-10 and the Metropolis chain
of App. G, plus the normaliser H of Sec. 4.1.

Target (eq. hk): over lattice points m != 0, P(m) = h(k) = exp(-k^2/(4 alpha^2))/H,
k = 2 pi (mx/Lx, my/Ly).

Proposal (App. G): m*_xi ~ N(0, (alpha L_xi)^2/(2 pi^2)), m_new = round(m*), which
is independent of the chain state, with probability
  q_xi(0) = erf(pi/(2 alpha L_xi)),
  q_xi(m) = 1/2 [erf(pi(2|m|+1)/(2 alpha L)) - erf(pi(2|m|-1)/(2 alpha L))]  (m != 0),
evaluated here as the equal difference of erfc values, which does not cancel
in the tails.  Acceptance (App. G) a = min(1, h(new) q(old) / (h(old) q(new))).

Readings of what App. G leaves open (the GPU sampler follows the same):
* random numbers: Philox4x32-10 (Salmon et al., SC'11) with key = (seed low,
  seed high) and counter = (draw index eta, step low, step high, stream), stream
  0 for the proposal's two normals (Box-Muller on two 53-bit uniforms) and
  stream 1 for the acceptance uniform; a 53-bit uniform from words (a, b) is
  ((a << 21) | (b >> 11)) + 0.5) * 2^-53;
* rounding: floor(m* + 1/2);
* a fresh chain per (seed, step): it starts at the first proposal that is not
  (0, 0) (eta0), then runs P*D Metropolis steps with proposals eta0+1, ...;
  the batch is the states after steps D, 2D, ..., P*D (thinning D, App. G);
* a proposal of (0, 0) has h = 0 and is always rejected.

The i.i.d. sampler (``sample_modes_iid``) is the exact alternative the chain
approximates: h factorises over the axes, so each draw inverts two
cumulative tables (Philox stream 2).

Pins (tests/test_oracle_sampler.py): Philox known-answer vectors published
with Random123 (tests/golden/philox4x32_10_kat.txt); a chi-square test of the
chain's frequencies against h; acceptance rate above 90% (App. G reports
over 90%); H by direct sum equals its Poisson closed form; for the i.i.d.
sampler a chi-square test against h (no correlation inflation), the
(0, 0) exclusion, and the marginal of m_x against the lattice sum.
"""

import math

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on Python ints: ctr 4 words, key 2 words."""
    c0, c1, c2, c3 = (int(v) & MASK for v in ctr)
    k0, k1 = (int(v) & MASK for v in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def philox4x32_10_vec(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox over numpy arrays of counters (uint64 holding 32-bit words)."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK
    c1 = np.broadcast_to(np.asarray(c1, dtype=np.uint64), c0.shape) & MASK
    c2 = np.broadcast_to(np.asarray(c2, dtype=np.uint64), c0.shape) & MASK
    c3 = np.broadcast_to(np.asarray(c3, dtype=np.uint64), c0.shape) & MASK
    k0 = np.uint64(k0 & MASK)
    k1 = np.uint64(k1 & MASK)
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    msk = np.uint64(MASK)
    s32 = np.uint64(32)
    for r in range(10):
        if r:
            k0 = np.uint64((int(k0) + W0) & MASK)
            k1 = np.uint64((int(k1) + W1) & MASK)
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> s32, p0 & msk
        hi1, lo1 = p1 >> s32, p1 & msk
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def _u53(a, b):
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    v = (a << np.uint64(21)) | (b >> np.uint64(11))
    return (v.astype(np.float64) + 0.5) * 2.0 ** -53


def proposals(seed, step, etas, alpha, Lx, Ly):
    """(mx, my, u_accept) for draw indices etas (numpy array)."""
    etas = np.asarray(etas, dtype=np.uint64)
    k0, k1 = seed & MASK, (seed >> 32) & MASK
    s0, s1 = step & MASK, (step >> 32) & MASK
    r0, r1, r2, r3 = philox4x32_10_vec(etas, s0, s1, 0, k0, k1)
    u1 = _u53(r0, r1)
    u2 = _u53(r2, r3)
    R = np.sqrt(-2.0 * np.log(u1))
    n1 = R * np.cos(2.0 * np.pi * u2)
    n2 = R * np.sin(2.0 * np.pi * u2)
    sx = alpha * Lx / (np.pi * math.sqrt(2.0))
    sy = alpha * Ly / (np.pi * math.sqrt(2.0))
    mx = np.floor(sx * n1 + 0.5).astype(np.int64)
    my = np.floor(sy * n2 + 0.5).astype(np.int64)
    a0, a1, _, _ = philox4x32_10_vec(etas, s0, s1, 1, k0, k1)
    return mx, my, _u53(a0, a1)


def _q1(m, aL):
    from scipy.special import erf, erfc
    m = abs(int(m))
    if m == 0:
        return float(erf(np.pi / (2.0 * aL)))
    return 0.5 * float(erfc(np.pi * (2 * m - 1) / (2.0 * aL)) - erfc(np.pi * (2 * m + 1) / (2.0 * aL)))


def weight(mx, my, alpha, Lx, Ly):
    """h(m)/q(m), unnormalised; 0 at m = (0, 0)."""
    if mx == 0 and my == 0:
        return 0.0
    kx = 2.0 * np.pi * mx / Lx
    ky = 2.0 * np.pi * my / Ly
    h = math.exp(-(kx * kx + ky * ky) / (4.0 * alpha * alpha))
    return h / (_q1(mx, alpha * Lx) * _q1(my, alpha * Ly))


def sample_modes(seed, step, P, alpha, Lx, Ly, thin=1, reserve=64):
    """The P modes of one step (see module docstring). Returns (P, 2) int array
    and the acceptance rate of the chain."""
    n = reserve + P * thin
    mx, my, u = proposals(seed, step, np.arange(n), alpha, Lx, Ly)
    eta0 = None
    for e in range(reserve):
        if mx[e] != 0 or my[e] != 0:
            eta0 = e
            break
    if eta0 is None:
        raise RuntimeError("no non-zero proposal among the reserved draws")
    cur = (int(mx[eta0]), int(my[eta0]))
    wcur = weight(cur[0], cur[1], alpha, Lx, Ly)
    out = []
    acc = 0
    for t in range(1, P * thin + 1):
        e = eta0 + t
        cand = (int(mx[e]), int(my[e]))
        wc = weight(cand[0], cand[1], alpha, Lx, Ly)
        if u[e] < wc / wcur:
            cur, wcur = cand, wc
            acc += 1
        if t % thin == 0:
            out.append(cur)
    return np.array(out, dtype=np.int64).reshape(-1, 2), acc / (P * thin)


def _axis_weights(alpha, L, mmax):
    """g(m) = exp(-(pi m / (alpha L))^2) for m = -mmax..mmax: the factor of
    h(k) = exp(-k^2/(4 alpha^2)) that belongs to one axis (k = 2 pi m / L)."""
    return [math.exp(-(math.pi * m / (alpha * L)) ** 2) for m in range(-mmax, mmax + 1)]


def _cdf(weights):
    """Cumulative sums in index order, divided by the total."""
    run = 0.0
    out = []
    for v in weights:
        run += v
        out.append(run)
    return np.array(out) / run


def iid_tables(alpha, Lx, Ly):
    """The three cumulative tables of the exact i.i.d. sampler: m_x from its
    marginal given m != (0, 0), m_y from g_y, and m_y from g_y without m_y = 0;
    axis ranges cover g >= 1e-18."""
    kmax = 2.0 * alpha * math.sqrt(math.log(1e18))
    mxm = int(math.ceil(kmax * Lx / (2 * math.pi)))
    mym = int(math.ceil(kmax * Ly / (2 * math.pi)))
    gx = _axis_weights(alpha, Lx, mxm)
    gy = _axis_weights(alpha, Ly, mym)
    zy = 0.0
    for v in gy:
        zy += v
    # P(m_x) = g_x(m_x) * (sum of g_y over the m_y allowed with this m_x)
    marg = [v * (zy - 1.0 if m == 0 else zy) for m, v in zip(range(-mxm, mxm + 1), gx)]
    nz = [0.0 if m == 0 else v for m, v in zip(range(-mym, mym + 1), gy)]
    return _cdf(marg), _cdf(gy), _cdf(nz), mxm, mym


def sample_modes_iid(seed, step, P, alpha, Lx, Ly):
    """P i.i.d. modes from h(k)/H over k != 0 (Sec. 4.1, eq. hk), an exact
    alternative to the chain of App. G: h factorises into one discrete Gaussian
    per axis, so draw m_x from its marginal given m != (0, 0), then m_y given
    m_x, each by inverting a cumulative table (the first entry >= u).  Draw i
    uses the two 53-bit uniforms of Philox block (counter (i, step, stream 2)).
    Returns a (P, 2) int array."""
    cx, cy, cy_nz, mxm, mym = iid_tables(alpha, Lx, Ly)
    k0, k1 = seed & MASK, (seed >> 32) & MASK
    r0, r1, r2, r3 = philox4x32_10_vec(np.arange(P, dtype=np.uint64), step & MASK,
                                       (step >> 32) & MASK, 2, k0, k1)
    ux = _u53(r0, r1)
    uy = _u53(r2, r3)
    out = np.zeros((P, 2), dtype=np.int64)
    for i in range(P):
        mx = int(np.searchsorted(cx, ux[i], side="left")) - mxm
        table = cy_nz if mx == 0 else cy
        my = int(np.searchsorted(table, uy[i], side="left")) - mym
        out[i] = (mx, my)
    return out


def H_value(Lx, Ly, alpha):
    from .lattice import H_direct
    return H_direct(Lx, Ly, alpha)
