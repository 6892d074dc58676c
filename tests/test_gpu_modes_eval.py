"""q2d_modes_eval: the k != 0 sum over a caller-given mode list.

* Small systems against the O(N) recursion (oracle O3) and the direct pair
  sums (oracle O2) with the k = 0 and self terms off and no j = i term, on
  random modes and weights: FP64 within 1e-10, FP32 within 1e-4.
* The exact-k reference of the N = 1e6 benchmark slab (all modes with
  e^{-k^2/4 alpha^2} >= 1e-16) is checked on 100 of its modes (500 with
  Q2D_SPOTCHECK_MODES=500), drawn at random with probability proportional to
  their weight, against the FP64 O(N) recursion (oracle O3) in FP64: the same
  kernels carry the whole list in q2d_long_range.
* Edge cases: an empty list, a (0, 0) entry (adds nothing), and agreement with
  the k != 0 pair part of q2d_rbm_step for its own sampled modes.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from _parity import assert_close  # noqa: E402

torch = pytest.importorskip("torch")

import paper_2403_01521_amd as q2d  # noqa: E402
import workloads as wl  # noqa: E402
from oracle import lattice, soewald2d  # noqa: E402
from oracle import recursion as o3  # noqa: E402


def dev(a, dt):
    return torch.tensor(np.asarray(a), dtype=dt, device="cuda")


def rel(a, b):
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def eval_modes(c, w, s, prec, modes, wt):
    dt = torch.float32 if prec == "fp32" else torch.float64
    plan = q2d.Plan(c["box"], c["alpha"], w, s, precision=prec, n_max=len(c["q"]))
    phi, F, E = plan.modes_eval(dev(c["pos"], dt), dev(c["q"], dt),
                                dev(np.asarray(modes, np.int32), torch.int32),
                                dev(np.asarray(wt, np.float64), torch.float64))
    torch.cuda.synchronize()
    out = (phi.double().cpu().numpy(), F.double().cpu().numpy(), float(E.cpu()[0]))
    plan.close()
    return out


def random_modes(rng, n, mmax):
    m = rng.integers(-mmax, mmax + 1, size=(n, 2))
    m[(m[:, 0] == 0) & (m[:, 1] == 0)] = [1, 2]
    return m


# FP32: the stated FP32 bar; a single mode of a small neutral system has a
# structure factor far below its terms, which lifts its relative error to ~1e-5
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
@pytest.mark.parametrize("nmodes", [1, 37, 100, 130])
def test_modes_eval_vs_pair_sums(soe_tables, prec, tol, nmodes):
    dtn = np.float32 if prec == "fp32" else np.float64
    c = wl.make_config(2, dtype=dtn, n_override=3000)
    w, s = soe_tables[16]
    rng = np.random.default_rng(100 + nmodes)
    modes = random_modes(rng, nmodes, 6)
    wt = rng.uniform(0.5, 2.0, nmodes) * np.pi / (c["box"][0] * c["box"][1])
    phi, F, E = eval_modes(c, w, s, prec, modes, wt)
    r = o3.long_range(c["pos"], c["q"], c["box"], c["alpha"], w, s, modes, wt,
                      include_self_pair=False, diag=0.0, nthreads=8)
    r0 = o3.long_range(c["pos"], c["q"], c["box"], c["alpha"], w, s, np.zeros((0, 2), int),
                       np.zeros(0), include_self_pair=False, diag=0.0, nthreads=1)
    ref_phi, ref_F, ref_U = r["phi"] - r0["phi"], r["F"] - r0["F"], r["U"] - r0["U"]
    print("modes_eval", prec, nmodes, rel(phi, ref_phi), rel(F, ref_F))
    assert_close(phi, ref_phi, tol)
    assert_close(F, ref_F, tol)
    assert abs(E - ref_U) < tol * abs(ref_U)
    # direct pair sums (O2) on sampled targets, k = 0 and self terms off
    tg = np.random.default_rng(7).choice(len(c["q"]), 4, replace=False)
    r2 = soewald2d.long_range(c["pos"], c["q"], c["box"], c["alpha"], w, s, modes, wt, targets=tg,
                              include_self_pair=False, diag=0.0, k0=False)
    assert_close(phi[tg], r2["phi"], tol)
    assert_close(F[tg], r2["F"], tol)


def test_modes_eval_edge_cases(soe_tables):
    c = wl.make_config(1, dtype=np.float64)
    w, s = soe_tables[16]
    # empty list: zero output
    phi, F, E = eval_modes(c, w, s, "fp64", np.zeros((0, 2), np.int32), np.zeros(0))
    assert np.all(phi == 0) and np.all(F == 0) and E == 0.0
    # a (0, 0) entry adds nothing
    modes = np.array([[1, 0], [0, 0], [2, -1]])
    wt = np.array([0.01, 5.0, 0.02])
    a = eval_modes(c, w, s, "fp64", modes, wt)
    b = eval_modes(c, w, s, "fp64", modes[[0, 2]], wt[[0, 2]])
    assert_close(a[0], b[0], 1e-13)
    assert_close(a[1], b[1], 1e-13)


def test_modes_eval_matches_rbm_pair_part(soe_tables):
    """rbm_step - k=0 part - diag constant - self = modes_eval on its modes."""
    c = wl.make_config(3, dtype=np.float64, n_override=5000)
    w, s = soe_tables[16]
    box, alpha = c["box"], c["alpha"]
    P = 100
    plan = q2d.Plan(box, alpha, w, s, precision="fp64", n_max=len(c["q"]), p_max=P)
    pos, q = dev(c["pos"], torch.float64), dev(c["q"], torch.float64)
    phi, F, E, modes = plan.rbm_step(pos, q, P, seed=5, step=9)
    H = lattice.H_direct(box[0], box[1], alpha)
    wt = torch.full((P,), np.pi / (box[0] * box[1]) * H / P, dtype=torch.float64, device="cuda")
    phi2, F2, E2 = plan.modes_eval(pos, q, modes, wt)
    torch.cuda.synchronize()
    info = plan.info()
    r0 = o3.long_range(c["pos"], c["q"], box, alpha, w, s, np.zeros((0, 2), int), np.zeros(0),
                       include_self_pair=False, diag=0.0, nthreads=1)
    qq = c["q"]
    phi_pair = phi.cpu().numpy() - r0["phi"] - qq * info["diag_rb"]
    F_pair = F.cpu().numpy() - r0["F"]
    assert_close(phi2.cpu().numpy(), phi_pair, 1e-10)
    assert_close(F2.cpu().numpy(), F_pair, 1e-10)
    plan.close()


def o3_chunked(c, w, s, modes, wt, chunk=25):
    """O3 over a long mode list in chunks (k = 0 part removed), printing progress."""
    box, alpha = c["box"], c["alpha"]
    z = np.zeros((0, 2), int)
    r0 = o3.long_range(c["pos"], c["q"], box, alpha, w, s, z, np.zeros(0),
                       include_self_pair=False, diag=0.0, nthreads=0)
    phi = np.zeros_like(r0["phi"])
    F = np.zeros_like(r0["F"])
    for i in range(0, len(modes), chunk):
        r = o3.long_range(c["pos"], c["q"], box, alpha, w, s, modes[i:i + chunk], wt[i:i + chunk],
                          include_self_pair=False, diag=0.0, nthreads=0)
        phi += r["phi"] - r0["phi"]
        F += r["F"] - r0["F"]
        print("  O3 modes %d/%d" % (min(i + chunk, len(modes)), len(modes)), flush=True)
    return phi, F


# 500 modes take O3 a few minutes on the host: opt in with Q2D_SPOTCHECK_MODES=500
SPOT_MODES = int(os.environ.get("Q2D_SPOTCHECK_MODES", "100"))


def test_exact_k_reference_spot_check_fullsize(soe_tables):
    """Random modes of the N = 1e6 exact-k list, FP64, against O3."""
    c = wl.make_config(3, dtype=np.float64)
    w, s = soe_tables[16]
    box, alpha = c["box"], c["alpha"]
    kc = 2 * alpha * np.sqrt(np.log(1e16))
    m, wt = soewald2d.exact_modes(box[0], box[1], alpha, kc)
    # drawn with probability proportional to the weight, so that the check is
    # not dominated by modes whose contribution is below the k = 0 part's
    # rounding (the reference subtracts O3's k = 0 part)
    sel = np.sort(np.random.default_rng(2024).choice(len(m), SPOT_MODES, replace=False,
                                                     p=wt / wt.sum()))
    phi, F, E = eval_modes(c, w, s, "fp64", m[sel], wt[sel])
    print("GPU done", flush=True)
    rphi, rF = o3_chunked(c, w, s, m[sel], wt[sel])
    eF = rel(F, rF)
    ephi = rel(phi, rphi)
    print("exact-k list (%d modes), %d sampled, N=1e6 FP64 vs O3: F %.3e phi %.3e"
          % (len(m), SPOT_MODES, eF, ephi))
    assert eF < 1e-10 and ephi < 1e-10
