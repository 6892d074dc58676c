"""Differentiation through the long-range sums (configuration 4: N = 1e5 charges
of valence 1 and 2, 200 x 200 x 8, alpha = 0.25, k_c = 1.6 -- 8,120 modes --,
M = 24).

* energy(): dE/dpos = -F and dE/dq = phi against central finite differences of
  the GPU energy (FP64, h = 1e-4) on 64 seeded particles at the full size, and
  against the analytic (exact, non-SOE) Ewald2D long-range force and potential
  of oracle O1 on a density-matched 1000-particle box;
* potential(): the adjoint scans (q2d_long_range_vjp / q2d_rbm_step_vjp) for
  random upstream weights g against the same vector-Jacobian product built from
  oracle O3 runs with sources q and g, and against finite differences of
  sum_i g_i phi_i; torch.autograd.gradcheck on a small system.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2403_01521_amd as q2d  # noqa: E402
import workloads as wl  # noqa: E402
from paper_2403_01521_amd import autograd as qa  # noqa: E402
from oracle import ewald2d, lattice, soewald2d  # noqa: E402
from oracle import recursion as o3  # noqa: E402


def dev(a, dt=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dt, device="cuda")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def small_system(n, seed, box=(20.0, 20.0, 8.0)):
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, q = wl.mixed_valence_ions(rng, n, box)
    return pos, q, box


@pytest.fixture(scope="module")
def config4(soe_tables):
    c = wl.make_config(4, dtype=np.float64)
    w, s = soe_tables[24]
    plan = q2d.Plan(c["box"], c["alpha"], w, s, kc=c["kc"], precision="fp64",
                    n_max=len(c["q"]))
    yield c, plan
    plan.close()


def test_energy_grad_vs_finite_differences_config4(config4):
    c, plan = config4
    pos = dev(c["pos"]).requires_grad_(True)
    q = dev(c["q"]).requires_grad_(True)
    E = qa.energy(plan, pos, q)
    E.backward()
    gpos = pos.grad.cpu().numpy()
    gq = q.grad.cpu().numpy()
    h = 1e-4
    Lz = c["box"][2]
    z = c["pos"][:, 2]
    ok = np.nonzero((z > 2 * h) & (z < Lz - 2 * h))[0]
    sel = np.random.default_rng(44).choice(ok, 64, replace=False)
    base_p = dev(c["pos"])
    base_q = dev(c["q"])

    def e_at(p, qq):
        _, _, e = plan.long_range(p, qq)
        return float(e.cpu()[0])

    fd_pos = np.zeros((64, 3))
    fd_q = np.zeros(64)
    for t, i in enumerate(sel):
        for d in range(3):
            p = base_p.clone()
            p[i, d] += h
            ep = e_at(p, base_q)
            p[i, d] -= 2 * h
            em = e_at(p, base_q)
            fd_pos[t, d] = (ep - em) / (2 * h)
        qq = base_q.clone()
        qq[i] += h
        ep = e_at(base_p, qq)
        qq[i] -= 2 * h
        em = e_at(base_p, qq)
        fd_q[t] = (ep - em) / (2 * h)
    e_pos = rel(gpos[sel], fd_pos)
    e_q = rel(gq[sel], fd_q)
    print("config4 N=1e5: dE/dpos vs FD %.3e, dE/dq vs FD %.3e" % (e_pos, e_q))
    assert e_pos < 1e-6
    assert e_q < 1e-6


def test_energy_grad_vs_analytic_ewald2d(soe_tables):
    pos, q, box = small_system(1000, 4001)
    w, s = soe_tables[24]
    alpha, kc = 0.25, 1.6
    plan = q2d.Plan(box, alpha, w, s, kc=kc, precision="fp64", n_max=len(q))
    p = dev(pos).requires_grad_(True)
    qq = dev(q).requires_grad_(True)
    E = qa.energy(plan, p, qq)
    E.backward()
    ref = ewald2d.long_range(pos, q, box, alpha, kc)
    e_f = rel(-p.grad.cpu().numpy(), ref["F"])
    e_phi = rel(qq.grad.cpu().numpy(), ref["phi"])
    e_E = abs(float(E.detach()) - ref["U"]) / abs(ref["U"])
    print("N=1000 autograd vs exact Ewald2D (O1): F %.3e phi %.3e E %.3e" % (e_f, e_phi, e_E))
    assert e_f < 1e-9 and e_phi < 1e-9 and e_E < 1e-9
    plan.close()


def oracle_vjp(pos, q, g, box, alpha, w, s, modes, wt, include_self_pair, diag):
    """dq = phi(g), dpos = -(g f(q) + q f(g)) from O3 runs with sources q and g."""
    rq = o3.long_range(pos, q, box, alpha, w, s, modes, wt, include_self_pair=include_self_pair,
                       diag=diag, nthreads=0)
    rg = o3.long_range(pos, g, box, alpha, w, s, modes, wt, include_self_pair=include_self_pair,
                       diag=diag, nthreads=0)
    fq = rq["F"] / q[:, None]
    fg = rg["F"] / g[:, None]
    return rg["phi"], -(g[:, None] * fq + q[:, None] * fg)


@pytest.fixture(scope="module")
def vjp_case(soe_tables):
    """Config-4 inputs at N = 2000 rounded to FP32 (exact in both precisions),
    random weights g, and the oracle's vector-Jacobian product."""
    c = wl.make_config(4, dtype=np.float32, n_override=2000)
    w, s = soe_tables[24]
    box, alpha, kc = c["box"], c["alpha"], c["kc"]
    g = np.random.default_rng(9).normal(size=len(c["q"])).astype(np.float32)
    m, wt = soewald2d.exact_modes(box[0], box[1], alpha, kc)
    ref = oracle_vjp(c["pos"].astype(np.float64), c["q"].astype(np.float64),
                     g.astype(np.float64), box, alpha, w, s, m, wt, True, 0.0)
    return c, g, ref


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_potential_vjp_exact_k(soe_tables, vjp_case, prec, tol):
    dt = torch.float64 if prec == "fp64" else torch.float32
    c, g, (dq_ref, dpos_ref) = vjp_case
    w, s = soe_tables[24]
    box, alpha, kc = c["box"], c["alpha"], c["kc"]
    plan = q2d.Plan(box, alpha, w, s, kc=kc, precision=prec, n_max=len(c["q"]))
    p = dev(c["pos"], dt).requires_grad_(True)
    qq = dev(c["q"], dt).requires_grad_(True)
    phi = qa.potential(plan, p, qq)
    phi.backward(dev(g, dt))
    e_q = rel(qq.grad.double().cpu().numpy(), dq_ref)
    e_p = rel(p.grad.double().cpu().numpy(), dpos_ref)
    print("exact-k VJP %s vs O3: dq %.3e dpos %.3e" % (prec, e_q, e_p))
    assert e_q < tol and e_p < tol
    plan.close()


def test_potential_vjp_random_batch(soe_tables):
    c = wl.make_config(4, dtype=np.float64, n_override=4000)
    w, s = soe_tables[24]
    box, alpha = c["box"], c["alpha"]
    P = 64
    g = np.random.default_rng(10).normal(size=len(c["q"]))
    plan = q2d.Plan(box, alpha, w, s, precision="fp64", n_max=len(c["q"]), p_max=P)
    p = dev(c["pos"]).requires_grad_(True)
    qq = dev(c["q"]).requires_grad_(True)
    phi = qa.potential(plan, p, qq, rb=(P, 77, 3))
    phi.backward(dev(g))
    _, _, _, modes = plan.rbm_step(dev(c["pos"]), dev(c["q"]), P, 77, 3)
    modes = modes.cpu().numpy()
    H = lattice.H_direct(box[0], box[1], alpha)
    D = soewald2d.diag_constant(box[0], box[1], alpha, w, s)
    wt = soewald2d.rb_weights(P, H, box[0], box[1])
    dq_ref, dpos_ref = oracle_vjp(c["pos"], c["q"], g, box, alpha, w, s, modes, wt, False, D)
    e_q = rel(qq.grad.cpu().numpy(), dq_ref)
    e_p = rel(p.grad.cpu().numpy(), dpos_ref)
    print("random-batch VJP vs O3: dq %.3e dpos %.3e" % (e_q, e_p))
    assert e_q < 1e-10 and e_p < 1e-10
    plan.close()


def test_potential_vjp_vs_finite_differences(soe_tables):
    pos, q, box = small_system(2000, 4002)
    w, s = soe_tables[24]
    alpha, kc = 0.25, 1.6
    plan = q2d.Plan(box, alpha, w, s, kc=kc, precision="fp64", n_max=len(q))
    g = np.random.default_rng(11).normal(size=len(q))
    p = dev(pos).requires_grad_(True)
    phi = qa.potential(plan, p, dev(q))
    phi.backward(dev(g))
    gpos = p.grad.cpu().numpy()
    gd = dev(g)

    def L(pp):
        ph, _, _ = plan.long_range(pp, dev(q))
        return float((ph * gd).sum())

    h = 1e-4
    ok = np.nonzero((pos[:, 2] > 2 * h) & (pos[:, 2] < box[2] - 2 * h))[0]
    sel = np.random.default_rng(12).choice(ok, 16, replace=False)
    base = dev(pos)
    fd = np.zeros((16, 3))
    for t, i in enumerate(sel):
        for d in range(3):
            pp = base.clone()
            pp[i, d] += h
            lp = L(pp)
            pp[i, d] -= 2 * h
            lm = L(pp)
            fd[t, d] = (lp - lm) / (2 * h)
    e = rel(gpos[sel], fd)
    print("VJP dpos vs FD of sum g*phi: %.3e" % e)
    assert e < 1e-6
    plan.close()


def test_gradcheck_small(soe_tables):
    pos, q, box = small_system(24, 4003, box=(6.0, 6.0, 3.0))
    w, s = soe_tables[24]
    plan = q2d.Plan(box, 0.8, w, s, kc=6.0, precision="fp64", n_max=len(q))
    p = dev(pos).requires_grad_(True)
    qq = dev(q).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: qa.potential(plan, a, b), (p, qq), eps=1e-6,
                                    atol=1e-7, rtol=1e-6)
    assert torch.autograd.gradcheck(lambda a, b: qa.energy(plan, a, b), (p, qq), eps=1e-6,
                                    atol=1e-7, rtol=1e-6)
    plan.close()
