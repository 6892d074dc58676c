"""Parity at the benchmark size: N = 1e6 slab (600 x 600 x 10, 10% surface
excess), alpha = 0.1, P = 100, M = 16, FP32 scans -- in the launch
configuration bench.py times.

* all particles against the FP64 O(N) recursion (oracle O3) on the same
  sampled modes: relative force RMS <= 1e-4 (the stated FP32 bar), reported
  for the total long-range force and for its k != 0 part alone (the strong
  k = 0 mean field of the surface excess could hide k != 0 error);
* 8 sampled particles against the direct pair sums (oracle O2);
* invariants that hold at any size: zero net force, and potential and force
  unchanged under a common shift of x, y (periodic) and z (kept in [0, Lz]);
* two more draws (other steps, other modes) against O3 on all particles;
* one draw with the model-reduced M = 10 SOE table (the accuracy of the
  M = 16 Talbot table with 6 exponent slots instead of 9) against O3.

Every comparison bounds each particle as well as the norm (tests/_parity.py).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from _parity import assert_close, per_particle  # noqa: E402

torch = pytest.importorskip("torch")

import paper_2403_01521_amd as q2d  # noqa: E402
import workloads as wl  # noqa: E402
from oracle import lattice, soewald2d  # noqa: E402
from oracle import recursion as o3  # noqa: E402

P = 100


@pytest.fixture(scope="module")
def fullsize(soe_tables):
    w, s = soe_tables[16]
    c = wl.make_config(3, dtype=np.float32)
    box, alpha = c["box"], c["alpha"]
    N = len(c["q"])
    plan = q2d.Plan(box, alpha, w, s, precision="fp32", n_max=N, p_max=P)
    pos = torch.tensor(c["pos"], device="cuda")
    q = torch.tensor(c["q"], device="cuda")
    phi, F, E, modes = plan.rbm_step(pos, q, P, seed=2024, step=17)
    torch.cuda.synchronize()
    out = dict(c=c, w=w, s=s, plan=plan, pos=pos, q=q, phi=phi.double().cpu().numpy(),
               F=F.double().cpu().numpy(), E=float(E.cpu()[0]), modes=modes.cpu().numpy())
    yield out
    plan.close()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_fullsize_vs_recursion_oracle(fullsize):
    f = fullsize
    c, w, s = f["c"], f["w"], f["s"]
    box, alpha = c["box"], c["alpha"]
    H = lattice.H_direct(box[0], box[1], alpha)
    D = soewald2d.diag_constant(box[0], box[1], alpha, w, s)
    wt = soewald2d.rb_weights(P, H, box[0], box[1])
    pos = c["pos"].astype(np.float64)
    q = c["q"].astype(np.float64)
    r = o3.long_range(pos, q, box, alpha, w, s, f["modes"], wt, include_self_pair=False,
                      diag=D, nthreads=16)
    # the k = 0 part alone (no modes) isolates the k != 0 force for a second check
    r0 = o3.long_range(pos, q, box, alpha, w, s, np.zeros((0, 2), int), np.zeros(0),
                       include_self_pair=False, diag=0.0, nthreads=1)
    eF = rel(f["F"], r["F"])
    eFk = rel(f["F"] - r0["F"], r["F"] - r0["F"])
    ephi = rel(f["phi"], r["phi"])
    eE = abs(f["E"] - r["U"]) / abs(r["U"])
    print("N=1e6 FP32 vs O3: F %.3e  F(k!=0) %.3e  phi %.3e  E %.3e; per particle F %.3e "
          "F(k!=0) %.3e phi %.3e" % (eF, eFk, ephi, eE, per_particle(f["F"], r["F"]),
                                     per_particle(f["F"] - r0["F"], r["F"] - r0["F"]),
                                     per_particle(f["phi"], r["phi"])))
    assert_close(f["F"], r["F"], 1e-4, "F")
    assert_close(f["F"] - r0["F"], r["F"] - r0["F"], 1e-4, "F k!=0")
    assert_close(f["phi"], r["phi"], 1e-4, "phi")
    assert eE <= 1e-4


def test_fullsize_sampled_pair_sums(fullsize):
    f = fullsize
    c, w, s = f["c"], f["w"], f["s"]
    box, alpha = c["box"], c["alpha"]
    H = lattice.H_direct(box[0], box[1], alpha)
    D = soewald2d.diag_constant(box[0], box[1], alpha, w, s)
    tg = np.random.default_rng(3).choice(len(c["q"]), 8, replace=False)
    r = soewald2d.rb(c["pos"].astype(np.float64), c["q"].astype(np.float64), box, alpha, w, s,
                     f["modes"], H, targets=tg, diag=D)
    eF = rel(f["F"][tg], r["F"])
    ephi = rel(f["phi"][tg], r["phi"])
    print("N=1e6 FP32 vs O2 on 8 particles: F %.3e phi %.3e" % (eF, ephi))
    assert_close(f["F"][tg], r["F"], 1e-4)
    assert_close(f["phi"][tg], r["phi"], 1e-4)


def test_fullsize_invariants(fullsize):
    f = fullsize
    c = f["c"]
    F = f["F"]
    # Newton's third law: the pair forces cancel; FP32 sum relative to the scale
    net = np.abs(F.sum(0)).max()
    scale = np.sqrt((F * F).sum() / len(F)) * np.sqrt(len(F))
    assert net < 1e-4 * scale, (net, scale)
    # shift every particle by the same vector: x, y periodic, z inside [0, Lz]
    box = c["box"]
    pos = c["pos"].astype(np.float64)
    sh = np.array([123.25, -47.5, -0.5 * pos[:, 2].min()])
    assert sh[2] < 0 or pos[:, 2].min() == 0.0
    pos2 = pos + sh
    assert pos2[:, 2].min() >= 0.0 and pos2[:, 2].max() <= box[2]
    pos2[:, 0] %= box[0]
    pos2[:, 1] %= box[1]
    p2 = torch.tensor(pos2.astype(np.float32), device="cuda")
    phi2, F2, E2, m2 = f["plan"].rbm_step(p2, f["q"], P, seed=2024, step=17)
    torch.cuda.synchronize()
    assert np.array_equal(m2.cpu().numpy(), f["modes"])
    assert_close(F2.double().cpu().numpy(), F, 1e-4)
    assert_close(phi2.double().cpu().numpy(), f["phi"], 1e-4)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("seed,step", [(7, 0), (99, 123456)])
def test_fullsize_more_draws_vs_recursion_oracle(fullsize, seed, step):
    """Other draws (other sampled modes) at N = 1e6 against O3 on all
    particles, per particle and in norm."""
    f = fullsize
    c, w, s = f["c"], f["w"], f["s"]
    box, alpha = c["box"], c["alpha"]
    print("draw seed=%d step=%d" % (seed, step), flush=True)
    phi, F, E, modes = f["plan"].rbm_step(f["pos"], f["q"], P, seed=seed, step=step)
    torch.cuda.synchronize()
    modes = modes.cpu().numpy()
    assert not np.array_equal(modes, f["modes"])
    H = lattice.H_direct(box[0], box[1], alpha)
    D = soewald2d.diag_constant(box[0], box[1], alpha, w, s)
    r = o3.long_range(c["pos"].astype(np.float64), c["q"].astype(np.float64), box, alpha, w, s,
                      modes, soewald2d.rb_weights(P, H, box[0], box[1]), include_self_pair=False,
                      diag=D, nthreads=16)
    Fg = F.double().cpu().numpy()
    pg = phi.double().cpu().numpy()
    e = assert_close(Fg, r["F"], 1e-4, "F")
    ep = assert_close(pg, r["phi"], 1e-4, "phi")
    print("draw (%d, %d): F %.3e (per particle %.3e) phi %.3e (%.3e)" % (seed, step, *e, *ep))
    assert abs(float(E.cpu()[0]) - r["U"]) <= 1e-4 * abs(r["U"])


@pytest.mark.timeout(900)
def test_fullsize_reduced_soe_vs_recursion_oracle(soe_tables):
    """The bench workload with the model-reduced M = 10 table: FP32 on all
    10^6 particles against O3 (FP64) on the same modes and table."""
    w, s = soe_tables["r10"]
    c = wl.make_config(3, dtype=np.float32)
    box, alpha = c["box"], c["alpha"]
    N = len(c["q"])
    print("reduced SOE M = 10, N = %d" % N, flush=True)
    plan = q2d.Plan(box, alpha, w, s, precision="fp32", n_max=N, p_max=P)
    phi, F, E, modes = plan.rbm_step(torch.tensor(c["pos"], device="cuda"),
                                     torch.tensor(c["q"], device="cuda"), P, seed=5, step=77)
    torch.cuda.synchronize()
    modes = modes.cpu().numpy()
    H = lattice.H_direct(box[0], box[1], alpha)
    D = soewald2d.diag_constant(box[0], box[1], alpha, w, s)
    r = o3.long_range(c["pos"].astype(np.float64), c["q"].astype(np.float64), box, alpha, w, s,
                      modes, soewald2d.rb_weights(P, H, box[0], box[1]), include_self_pair=False,
                      diag=D, nthreads=16)
    e = assert_close(F.double().cpu().numpy(), r["F"], 1e-4, "F")
    ep = assert_close(phi.double().cpu().numpy(), r["phi"], 1e-4, "phi")
    print("reduced SOE: F %.3e (per particle %.3e) phi %.3e (%.3e)" % (*e, *ep))
    assert abs(float(E.cpu()[0]) - r["U"]) <= 1e-4 * abs(r["U"])
    plan.close()
