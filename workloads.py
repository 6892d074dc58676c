"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the method: it only draws charges and
positions.  Both the GPU library's callers and the CPU oracle consume what it
returns.  Positions are drawn in FP64 with NumPy's PCG64 and then rounded to
the requested dtype; callers hand the rounded values to both sides, so input
quantisation is never counted as error.

The paper's workloads are synthetic uniform ion boxes with charges +-1
(Sec. 5: e.g. 50 cations + 50 anions in a box; 1:1 electrolytes); there is no
public dataset.  The configurations below follow that recipe:

  1  N=100, 50 x (+1) and 50 x (-1), uniform in [0,20)^2 x [0,5];
     alpha=0.4, r_c=10, k_c=3.4, M=16                       (plain Ewald2D check)
  2  N=1e4, +-1 neutral, uniform in [0,60)^2 x [0,10];
     alpha=0.25, k_c=1.6, M=24                              (exact-k SOE)
  3  N=1e6, +-1 neutral in [0,600)^2 x [0,10] with a surface excess: 5e4 of the
     5e5 cations uniform in z in [0,1] and 5e4 of the 5e5 anions uniform in
     z in [9,10], the rest uniform in [0,10]; alpha=0.1, P=100, M=16
                                                           (random batch step)
  4  N=1e5, |q| in {1,2}, random signs, neutral, [0,200)^2 x [0,8];
     alpha=0.25, k_c=1.6, M=24
"""

import numpy as np

SEED_BASE = 20240302


def rng_for(idx):
    return np.random.Generator(np.random.PCG64(SEED_BASE + int(idx)))


def _shuffle(rng, pos, q):
    p = rng.permutation(len(q))
    return pos[p], q[p]


def uniform_ions(rng, n_pos, n_neg, box):
    Lx, Ly, Lz = box
    n = n_pos + n_neg
    pos = np.empty((n, 3))
    pos[:, 0] = rng.uniform(0.0, Lx, n)
    pos[:, 1] = rng.uniform(0.0, Ly, n)
    pos[:, 2] = rng.uniform(0.0, Lz, n)
    q = np.concatenate([np.ones(n_pos), -np.ones(n_neg)])
    return _shuffle(rng, pos, q)


def surface_excess_ions(rng, n_pos, n_neg, box, n_excess, layer):
    """+-1 ions uniform in the box except n_excess cations in z in [0, layer]
    and n_excess anions in z in [Lz - layer, Lz]."""
    Lx, Ly, Lz = box
    n = n_pos + n_neg
    pos = np.empty((n, 3))
    pos[:, 0] = rng.uniform(0.0, Lx, n)
    pos[:, 1] = rng.uniform(0.0, Ly, n)
    z = np.empty(n)
    z[:n_excess] = rng.uniform(0.0, layer, n_excess)
    z[n_excess:n_pos] = rng.uniform(0.0, Lz, n_pos - n_excess)
    z[n_pos:n_pos + n_excess] = rng.uniform(Lz - layer, Lz, n_excess)
    z[n_pos + n_excess:] = rng.uniform(0.0, Lz, n_neg - n_excess)
    pos[:, 2] = z
    q = np.concatenate([np.ones(n_pos), -np.ones(n_neg)])
    return _shuffle(rng, pos, q)


def mixed_valence_ions(rng, n, box):
    """|q| in {1, 2} iid, signs half and half, magnitudes rebalanced to zero net
    charge (n even): while the net charge is positive, a +2 becomes +1 or a -1
    becomes -2 (and conversely), visiting particles in a random order."""
    Lx, Ly, Lz = box
    pos = np.empty((n, 3))
    pos[:, 0] = rng.uniform(0.0, Lx, n)
    pos[:, 1] = rng.uniform(0.0, Ly, n)
    pos[:, 2] = rng.uniform(0.0, Lz, n)
    mag = rng.integers(1, 3, n).astype(np.float64)
    sign = np.ones(n)
    sign[rng.permutation(n)[: n // 2]] = -1.0
    q = mag * sign
    net = q.sum()
    for j in rng.permutation(n):
        if net == 0:
            break
        s = np.sign(net)
        # lower the magnitude of a charge of the net's sign, or raise one of the other
        if q[j] == 2 * s or q[j] == -s:
            q[j] -= s
            net -= s
    if net != 0:
        raise RuntimeError("could not neutralise")
    return pos, q


CONFIGS = {
    1: dict(name="ewald2d_N100", box=(20.0, 20.0, 5.0), alpha=0.4, rc=10.0, kc=3.4, M=16),
    2: dict(name="exactk_N1e4", box=(60.0, 60.0, 10.0), alpha=0.25, rc=None, kc=1.6, M=24),
    3: dict(name="rbm_N1e6", box=(600.0, 600.0, 10.0), alpha=0.1, rc=None, kc=None, M=16, P=100),
    4: dict(name="grad_N1e5", box=(200.0, 200.0, 8.0), alpha=0.25, rc=None, kc=1.6, M=24),
    5: dict(name="replicas_R256", R=256, n_range=(1000, 20000), Lz=6.0, density=0.05,
            L_range=(30.0, 150.0), alpha=0.3, M=16, P=64),
}


def make_replicas(R=None, n_range=None, dtype=np.float64):
    """Configuration 5: R independent +-1 systems, N_r log-uniform in n_range
    (rounded to even), Lx = Ly = clamp(sqrt(N_r / (density Lz)), L_range),
    uniform in [0, L)^2 x [0, Lz].  Returns dict(pos, q (concatenated by
    replica), boxes (R x 3), counts, alpha, M, P)."""
    c = dict(CONFIGS[5])
    rng = rng_for(5)
    R = R or c["R"]
    lo, hi = n_range or c["n_range"]
    counts = np.exp(rng.uniform(np.log(lo), np.log(hi), R))
    counts = (2 * np.round(counts / 2)).astype(np.int64)
    Lz = c["Lz"]
    L = np.clip(np.sqrt(counts / (c["density"] * Lz)), *c["L_range"])
    boxes = np.stack([L, L, np.full(R, Lz)], axis=1)
    pos, q = [], []
    for r in range(R):
        p, qq = uniform_ions(rng, counts[r] // 2, counts[r] // 2, tuple(boxes[r]))
        pos.append(p)
        q.append(qq)
    c.update(pos=np.concatenate(pos).astype(dtype), q=np.concatenate(q).astype(dtype),
             boxes=boxes, counts=counts, R=R)
    return c


def make_config(idx, dtype=np.float64, n_override=None):
    """Inputs of a numbered configuration: dict(pos, q, box, alpha, rc, kc, M[, P])."""
    c = dict(CONFIGS[idx])
    rng = rng_for(idx)
    box = c["box"]
    if idx == 1:
        n = n_override or 100
        pos, q = uniform_ions(rng, n // 2, n // 2, box)
    elif idx == 2:
        n = n_override or 10000
        pos, q = uniform_ions(rng, n // 2, n // 2, box)
    elif idx == 3:
        n = n_override or 1000000
        pos, q = surface_excess_ions(rng, n // 2, n // 2, box, n // 20, 1.0)
    elif idx == 4:
        n = n_override or 100000
        pos, q = mixed_valence_ions(rng, n, box)
    else:
        raise KeyError(idx)
    c["pos"] = pos.astype(dtype)
    c["q"] = q.astype(dtype)
    return c


def random_system(n, box, seed, dtype=np.float64, z_values=None):
    """n (even) +-1 ions uniform in box, optionally with z drawn from z_values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, q = uniform_ions(rng, n // 2, n - n // 2, box)
    if n % 2:
        q[-1] = 0.0
    if z_values is not None:
        pos[:, 2] = rng.choice(np.asarray(z_values, dtype=np.float64), n)
    return pos.astype(dtype), q.astype(dtype)


def square_ionic_cell(a, z0):
    """Four ions of the 2-D square ionic lattice (spacing a) in a 2a x 2a cell,
    all at height z0: + at (0,0), - at (a,0), - at (0,a), + at (a,a)."""
    pos = np.array([[0.0, 0.0, z0], [a, 0.0, z0], [0.0, a, z0], [a, a, z0]])
    q = np.array([1.0, -1.0, -1.0, 1.0])
    return pos, q
