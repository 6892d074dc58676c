"""FP32 aggregate pass on the fp16 matrix cores (split operands).

The FP32 plans compute the segment aggregates with every operand carried as two
fp16 halves and the sources scaled per segment by a power of two.  These tests
pin that arithmetic against relations that hold exactly and against the FP64
path (which does not use fp16):

* charge scaling: q -> s q multiplies phi by s and F, E by s^2 (the method is
  linear in the sources); s = 1e6 takes |q| far past the fp16 range, s = 1e-7
  puts every source in the fp16 subnormal range without the scaling.  Both FP32
  runs (rescaled) must match the FP64 oracle (O3) as closely as each other;
* mixed magnitudes (charges 1 and 1000 in one segment) and two thin slabs with a
  wide empty gap (long segment spans, large decay phases): FP32 against the
  FP64 O(N) recursion of the oracle (O3) on the same modes within 2e-5, per
  particle as well as in norm; for mixed magnitudes also over the unit
  charges alone (whose sources sit near the fp16 normal range after the
  per-segment scaling, and whose forces the +-1000 ions dominate in the norm);
* the Taylor columns of the beta = k term: segments on both sides of the
  |k|max x span <= 0.4 threshold in one launch, against O3 segment by segment.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from _parity import assert_close, rel as prel  # noqa: E402

torch = pytest.importorskip("torch")

import paper_2403_01521_amd as q2d  # noqa: E402
import workloads as wl  # noqa: E402
from oracle import lattice, soewald2d  # noqa: E402
from oracle import recursion as o3  # noqa: E402

P = 64


def dev(a, dt):
    return torch.tensor(np.asarray(a), dtype=dt, device="cuda")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def step(box, alpha, w, s, pos, q, prec, seed=21, stepno=3):
    dt = torch.float32 if prec == "fp32" else torch.float64
    plan = q2d.Plan(box, alpha, w, s, precision=prec, n_max=len(q), p_max=P)
    phi, F, E, modes = plan.rbm_step(dev(pos, dt), dev(q, dt), P, seed, stepno)
    torch.cuda.synchronize()
    out = (phi.double().cpu().numpy(), F.double().cpu().numpy(), float(E.cpu()[0]),
           modes.cpu().numpy())
    plan.close()
    return out


@pytest.mark.parametrize("scale", [1e6, 1e-7])
def test_charge_scaling(soe_tables, scale):
    c = wl.make_config(3, dtype=np.float32, n_override=6000)
    w, s = soe_tables[16]
    q = c["q"].astype(np.float32)
    qs = (q.astype(np.float64) * scale).astype(np.float32)
    # the exact scale factor after FP32 rounding of the charges
    ratio = float(np.median(qs.astype(np.float64) / q.astype(np.float64)))
    phi1, F1, E1, m1 = step(c["box"], c["alpha"], w, s, c["pos"], q, "fp32")
    phi2, F2, E2, m2 = step(c["box"], c["alpha"], w, s, c["pos"], qs, "fp32")
    box, alpha = c["box"], c["alpha"]
    assert np.array_equal(m1, m2)
    H = lattice.H_direct(box[0], box[1], alpha)
    D = soewald2d.diag_constant(box[0], box[1], alpha, w, s)
    r = o3.long_range(c["pos"].astype(np.float64), q.astype(np.float64), box, alpha, w, s, m1,
                      soewald2d.rb_weights(P, H, box[0], box[1]), include_self_pair=False,
                      diag=D, nthreads=8)
    phi0, F0, E0 = r["phi"], r["F"], r["U"]
    assert np.all(np.isfinite(phi2)) and np.all(np.isfinite(F2))
    # each FP32 run against the FP64 oracle on the same modes (two independent
    # FP32 roundings are not compared with each other)
    e1 = (rel(phi1, phi0), rel(F1, F0), abs(E1 - E0) / abs(E0))
    e2 = (rel(phi2 / ratio, phi0), rel(F2 / ratio**2, F0), abs(E2 / ratio**2 - E0) / abs(E0))
    print("scale %g: unscaled phi %.2e F %.2e E %.2e | scaled phi %.2e F %.2e E %.2e"
          % ((scale,) + e1 + e2))
    for a, b in zip(e1, e2):
        assert a < 3e-5 and b < 3e-5
        assert b < 2 * a + 1e-5
    assert_close(phi2 / ratio, phi0, 3e-5, "phi scaled")
    assert_close(F2 / ratio**2, F0, 3e-5, "F scaled")

def two_slabs(rng, n, box):
    """Half the ions in z in [0, 0.05 Lz], half in [0.95 Lz, Lz]: the middle is empty."""
    pos, q = wl.uniform_ions(rng, n // 2, n - n // 2, tuple(box))
    pos = pos.reshape(-1, 3)
    z = pos[:, 2] / box[2]
    pos[:, 2] = np.where(np.arange(len(z)) % 2 == 0, 0.05 * z, 1.0 - 0.05 * z) * box[2]
    return pos, q


def mixed_charges(rng, n, box):
    """Unit ions with every 97th charge scaled to +-1000 (pairs keep the sum zero)."""
    pos, q = wl.uniform_ions(rng, n // 2, n - n // 2, tuple(box))
    q = q.copy()
    idx = np.arange(0, n - 1, 97)
    q[idx] *= 1000.0
    # restore neutrality with the opposite big charge on the next particle
    q[idx + 1] = -q[idx]
    q[-1] -= q.sum()
    return pos.reshape(-1, 3), q


@pytest.mark.parametrize("maker", [two_slabs, mixed_charges])
def test_fp32_vs_fp64_hard_inputs(soe_tables, maker):
    rng = np.random.Generator(np.random.PCG64(777))
    box = (40.0, 40.0, 8.0)
    pos, q = maker(rng, 5000, box)
    pos32, q32 = pos.astype(np.float32), q.astype(np.float32)
    w, s = soe_tables[16]
    phi32, F32, E32, m32 = step(box, 0.3, w, s, pos32, q32, "fp32")
    alpha = 0.3
    H = lattice.H_direct(box[0], box[1], alpha)
    D = soewald2d.diag_constant(box[0], box[1], alpha, w, s)
    r = o3.long_range(pos32.astype(np.float64), q32.astype(np.float64), box, alpha, w, s, m32,
                      soewald2d.rb_weights(P, H, box[0], box[1]), include_self_pair=False,
                      diag=D, nthreads=8)
    phi64, F64, E64 = r["phi"], r["F"], r["U"]
    print("%s: phi %.2e F %.2e E %.2e" % (maker.__name__, rel(phi32, phi64), rel(F32, F64),
                                         abs(E32 - E64) / abs(E64)))
    assert_close(phi32, phi64, 2e-5, "phi")
    assert_close(F32, F64, 2e-5, "F")
    assert abs(E32 - E64) < 2e-5 * abs(E64)
    unit = np.abs(q32) == 1.0
    if not unit.all():
        print("  unit charges only: phi %.2e F %.2e" % (prel(phi32[unit], phi64[unit]),
                                                        prel(F32[unit], F64[unit])))
        assert_close(phi32[unit], phi64[unit], 2e-5, "phi |q|=1")
        assert_close(F32[unit], F64[unit], 2e-5, "F |q|=1")


def test_taylor_columns_threshold(soe_tables):
    """The beta = k aggregate of a segment goes through Taylor columns in
    u = t / Delta when (largest |k| of the launch) x (segment span Delta) is at
    most 0.4, and through per-particle exponentials otherwise.  Eight segments
    of 512 particles with spans 0.05 ... 6 in units of 1 / |k|max (0.39 and
    0.41 on either side of the threshold) in one launch of a fixed mode list
    whose largest |k| is 1: FP32 against the FP64 O(N) recursion (O3), per
    particle and in norm, and segment by segment."""
    box = (20 * np.pi, 20 * np.pi, 40.0)  # k = (mx, my) / 10
    alpha = 0.5
    w, s = soe_tables[16]
    rng = np.random.default_rng(1234)
    spans = [0.05, 0.2, 0.39, 0.41, 0.6, 1.5, 3.0, 6.0]
    S = 512
    zs, z0 = [], 1.0
    for d in spans:
        z = z0 + d * rng.uniform(0.0, 1.0, S)
        z[0], z[-1] = z0, z0 + d  # the segment's span is exactly d
        zs.append(np.sort(z))
        z0 += d + 1.0
    assert z0 < box[2]
    z = np.concatenate(zs)
    n = len(z)
    pos = np.stack([rng.uniform(0, box[0], n), rng.uniform(0, box[1], n), z], axis=1)
    q = rng.permutation(np.repeat([1.0, -1.0], n // 2))  # neutral
    pos32, q32 = pos.astype(np.float32), q.astype(np.float32)
    modes = np.array([[10, 0]] + [list(m) for m in rng.integers(-7, 8, size=(95, 2))
                                  if (m[0], m[1]) != (0, 0)])
    kmag = np.hypot(modes[:, 0], modes[:, 1]) / 10.0
    assert kmag.max() == 1.0
    wt = rng.uniform(0.5, 2.0, len(modes)) * np.pi / (box[0] * box[1])
    plan = q2d.Plan(box, alpha, w, s, precision="fp32", n_max=n)
    phi, F, E = plan.modes_eval(dev(pos32, torch.float32), dev(q32, torch.float32),
                                dev(modes.astype(np.int32), torch.int32),
                                dev(wt, torch.float64))
    torch.cuda.synchronize()
    phi, F = phi.double().cpu().numpy(), F.double().cpu().numpy()
    plan.close()
    p64, q64 = pos32.astype(np.float64), q32.astype(np.float64)
    r = o3.long_range(p64, q64, box, alpha, w, s, modes, wt, include_self_pair=False, diag=0.0,
                      nthreads=8)
    r0 = o3.long_range(p64, q64, box, alpha, w, s, np.zeros((0, 2), int), np.zeros(0),
                       include_self_pair=False, diag=0.0, nthreads=1)
    ref_phi, ref_F = r["phi"] - r0["phi"], r["F"] - r0["F"]
    print("taylor threshold: phi %.2e F %.2e" % (rel(phi, ref_phi), rel(F, ref_F)))
    assert_close(phi, ref_phi, 2e-5, "phi")
    assert_close(F, ref_F, 2e-5, "F")
    # the sorted order is the input order here: segment g is rows g S .. (g + 1) S
    scale = np.sqrt(np.mean(np.sum(ref_F**2, axis=1)))
    for g, d in enumerate(spans):
        sl = slice(g * S, (g + 1) * S)
        err = np.abs(F[sl] - ref_F[sl]).max() / scale
        print("  span %.2f: max |dF| / rms F = %.2e" % (d, err))
        assert err < 5e-5, (d, err)
