"""Charged walls (q2d_slab) and the Langevin step (q2d_langevin_step) against
the oracle (oracle/slabs.py), and a short molecular-dynamics run that uses
every force term of Alg. 2 (random-batch long range, short range, walls)
with the Langevin step of Sec. 4.3.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from _parity import assert_close  # noqa: E402

torch = pytest.importorskip("torch")

import paper_2403_01521_amd as q2d  # noqa: E402
import workloads as wl  # noqa: E402
from oracle import slabs  # noqa: E402


def dev(a, dt):
    return torch.tensor(np.asarray(a), dtype=dt, device="cuda")


def host(t):
    return t.double().cpu().numpy()


PREC = [("fp64", torch.float64, np.float64, 1e-12), ("fp32", torch.float32, np.float32, 2e-6)]


@pytest.mark.parametrize("prec,dt,dtn,tol", PREC)
def test_uniform_walls(soe_tables, prec, dt, dtn, tol):
    box = (30.0, 20.0, 6.0)
    w, s = soe_tables[8]
    pos, q = wl.random_system(3001, box, seed=12, dtype=dtn)
    plan = q2d.Plan(box, 0.5, w, s, precision=prec, n_max=len(q))
    A = box[0] * box[1]
    sb, st = 0.013, -0.021
    phi, F, E = plan.slab(dev(pos, dt), dev(q, dt), sb * A, st * A)
    torch.cuda.synchronize()
    r = slabs.slab_uniform(pos, q, box, sb, st)
    assert_close(host(phi), r["phi"], tol, "phi")
    assert_close(host(F), r["F"], tol, "F")
    assert abs(float(E.cpu()[0]) - r["U"]) <= tol * np.abs(q * r["phi"]).sum()
    plan.close()


@pytest.mark.parametrize("prec,dt,dtn,tol", PREC)
def test_wall_series(soe_tables, prec, dt, dtn, tol):
    box = (25.0, 18.0, 5.0)
    w, s = soe_tables[8]
    pos, q = wl.random_system(2000, box, seed=13, dtype=dtn)
    rng = np.random.Generator(np.random.PCG64(5))
    half = np.array([[1, 0], [0, 1], [1, 1], [2, -1], [3, 2], [0, 4]])
    modes = np.concatenate([half, -half])
    cb = rng.normal(size=len(half)) + 1j * rng.normal(size=len(half))
    ct = rng.normal(size=len(half)) + 1j * rng.normal(size=len(half))
    cb = np.concatenate([cb, np.conj(cb)])  # real densities: sig(-k) = conj sig(k)
    ct = np.concatenate([ct, np.conj(ct)])
    plan = q2d.Plan(box, 0.5, w, s, precision=prec, n_max=len(q))
    phi, F, E = plan.slab(dev(pos, dt), dev(q, dt), 0.4, -0.9, dev(modes, torch.int32),
                          dev(cb, torch.complex128), dev(ct, torch.complex128))
    torch.cuda.synchronize()
    r = slabs.slab_series(pos, q, box, modes, cb, ct, 0.4, -0.9)
    assert_close(host(phi), r["phi"], tol, "phi")
    assert_close(host(F), r["F"], tol, "F")
    plan.close()


@pytest.mark.parametrize("prec,dt,dtn,tol", PREC)
def test_langevin_step(soe_tables, prec, dt, dtn, tol):
    box = (20.0, 15.0, 4.0)
    w, s = soe_tables[8]
    n = 5000
    rng = np.random.Generator(np.random.PCG64(8))
    pos, _ = wl.random_system(n, box, seed=14)
    pos[:5, 2] = [0.001, box[2] - 0.001, 0.0, box[2], 2.0]  # near and on the walls
    mom = rng.normal(size=(n, 3))
    mom[:2, 2] = [-3.0, 3.0]  # these two cross a wall
    mass = rng.uniform(0.5, 2.0, n)
    F1 = rng.normal(size=(n, 3))
    F2 = rng.normal(size=(n, 3))
    pos, mom, mass, F1, F2 = (a.astype(dtn) for a in (pos, mom, mass, F1, F2))
    plan = q2d.Plan(box, 0.5, w, s, precision=prec, n_max=n)
    P, M, m = dev(pos, dt), dev(mom, dt), dev(mass, dt)
    step_dt, gamma, kT = 0.01, 0.7, 1.3
    plan.langevin_step(P, M, [dev(F1, dt)], step_dt, gamma, kT, seed=99, step=7, stage=0, mass=m)
    plan.langevin_step(P, M, [dev(F2, dt)], step_dt, gamma, kT, seed=99, step=7, stage=1, mass=m)
    torch.cuda.synchronize()
    rp, rm = slabs.baoab_first(pos, mom, mass, F1, box, step_dt, gamma, kT, 99, 7)
    rm = slabs.baoab_second(rm, F2, step_dt)
    assert_close(host(P), rp, tol, "pos")
    assert_close(host(M), rm, tol, "mom")
    assert float(P[:, 2].min()) >= 0.0 and float(P[:, 2].max()) <= box[2]
    plan.close()


def test_short_md_run_holds_temperature(soe_tables):
    """A weakly charged neutral system between uniformly charged walls, driven
    by the random-batch long-range, short-range and wall forces through the
    Langevin step: the particles stay in the slab and the kinetic temperature
    settles at kT (within its statistical error)."""
    box = (40.0, 40.0, 8.0)
    n = 4000
    pos, q = wl.random_system(n, box, seed=15)
    q *= 0.1
    w, s = soe_tables[8]
    alpha = (n / np.prod(box)) ** (1 / 3)  # eq. 59
    rc = 4.0 / alpha                        # eq. rckc with s = 4
    plan = q2d.Plan(box, alpha, w, s, rc=rc, precision="fp64", n_max=n, p_max=32)
    A = box[0] * box[1]
    P, Q = dev(pos, torch.float64), dev(q, torch.float64)
    # momenta from the Maxwell-Boltzmann law at kT (unit masses)
    Mo = dev(np.random.Generator(np.random.PCG64(16)).normal(size=(n, 3)), torch.float64)
    kT, gamma, dt, steps = 1.0, 1.0, 0.01, 300

    def forces(step):
        _, Fl, _, _ = plan.rbm_step(P, Q, 32, seed=4, step=step)
        _, Fs, _ = plan.short_range(P, Q)
        _, Fw, _ = plan.slab(P, Q, 0.001 * A, -0.001 * A)
        return [Fl, Fs, Fw]

    F = forces(0)
    temps = []
    for t in range(steps):
        plan.langevin_step(P, Mo, F, dt, gamma, kT, seed=21, step=t, stage=0)
        F = forces(t + 1)
        plan.langevin_step(P, Mo, F, dt, gamma, kT, seed=21, step=t, stage=1)
        if t >= steps // 2:
            temps.append(float((Mo * Mo).sum()) / (3 * n))
    torch.cuda.synchronize()
    Tm = float(np.mean(temps))
    print("kinetic temperature %.4f (kT = %.1f)" % (Tm, kT))
    assert bool(torch.isfinite(P).all()) and bool(torch.isfinite(Mo).all())
    assert float(P[:, 2].min()) >= 0.0 and float(P[:, 2].max()) <= box[2]
    assert abs(Tm - kT) < 0.05 * kT
    plan.close()
