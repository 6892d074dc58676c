"""The allocation-free random-batch step (q2d_rbm_step_noalloc) against the
allocating one (q2d_rbm_step), through the C ABI.

Both run the same kernels on the same inputs, so every output must agree bit
for bit (the reductions have a fixed order); the only difference is where the
call's scratch lives (the library's static per-device array instead of the
plan's buffers).  Two calls in a row, the second with a smaller input, check
that a call does not depend on what the previous one left in the array; an
allocating call in between checks that the plan's own buffers are untouched.
A size whose scratch exceeds the array is refused with Q2D_ECAPACITY.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2403_01521_amd as q2d  # noqa: E402
import workloads as wl  # noqa: E402


def inputs(n, dtn, dt):
    c = wl.make_config(3, dtype=dtn, n_override=n)
    return (c, torch.tensor(c["pos"], dtype=dt, device="cuda"),
            torch.tensor(c["q"], dtype=dt, device="cuda"))


def same(a, b):
    a = [x.cpu() for x in a]
    b = [x.cpu() for x in b]
    for x, y, name in zip(a, b, ("phi", "F", "E", "modes")):
        assert x.shape == y.shape, name
        assert torch.equal(x, y), (name, float((x.double() - y.double()).abs().max()))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_matches_rbm_step(soe_tables, prec):
    dtn = np.float32 if prec == "fp32" else np.float64
    dt = torch.float32 if prec == "fp32" else torch.float64
    w, s = soe_tables[16]
    c, pos1, q1 = inputs(40000, dtn, dt)
    _, pos2, q2 = inputs(4097, dtn, dt)
    plan = q2d.Plan(c["box"], c["alpha"], w, s, precision=prec, n_max=40000, p_max=128)
    # first call: the larger input; the outputs are preallocated by the caller
    P1 = 100
    out1 = (torch.empty(40000, dtype=dt, device="cuda"),
            torch.empty((40000, 3), dtype=dt, device="cuda"),
            torch.empty(1, dtype=torch.float64, device="cuda"),
            torch.empty((P1, 2), dtype=torch.int32, device="cuda"))
    a1 = plan.rbm_step_noalloc(pos1, q1, P1, seed=5, step=3, out=out1)
    r1 = plan.rbm_step(pos1, q1, P1, seed=5, step=3)
    torch.cuda.synchronize()
    print(prec, "call 1: N = 40000, P = 100")
    same(a1, r1)
    # second call, smaller input, other modes (P = 37: three bands)
    a2 = plan.rbm_step_noalloc(pos2, q2, 37, seed=6, step=11)
    torch.cuda.synchronize()
    r2 = plan.rbm_step(pos2, q2, 37, seed=6, step=11)
    torch.cuda.synchronize()
    print(prec, "call 2: N = 4097, P = 37")
    same(a2, r2)
    # the larger input again after an allocating call: the plan's buffers and
    # the static array do not disturb each other
    a3 = plan.rbm_step_noalloc(pos1, q1, P1, seed=5, step=3)
    torch.cuda.synchronize()
    same(a3, r1)
    plan.close()


def test_noalloc_edge_cases(soe_tables):
    w, s = soe_tables[16]
    c, pos, q = inputs(2, np.float32, torch.float32)
    plan = q2d.Plan(c["box"], c["alpha"], w, s, precision="fp32", n_max=600000, p_max=100)
    # N = 0 writes E = 0; N = 1 and 2 agree with the allocating call
    e0 = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    m0 = torch.empty((4, 2), dtype=torch.int32, device="cuda")
    empty = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    plan.rbm_step_noalloc(empty, torch.empty(0, dtype=torch.float32, device="cuda"), 4, seed=1,
                          step=0, out=(torch.empty(0, device="cuda"),
                                       torch.empty((0, 3), device="cuda"), e0, m0))
    torch.cuda.synchronize()
    assert float(e0.cpu()[0]) == 0.0
    for n in (1, 2):
        a = plan.rbm_step_noalloc(pos[:n].contiguous(), q[:n].contiguous(), 4, seed=2, step=n)
        r = plan.rbm_step(pos[:n].contiguous(), q[:n].contiguous(), 4, seed=2, step=n)
        torch.cuda.synchronize()
        same(a, r)
    # beyond the static array: refused before any work, the plan still works
    _, posb, qb = inputs(600000, np.float32, torch.float32)
    with pytest.raises(q2d.Q2DError) as ei:
        plan.rbm_step_noalloc(posb, qb, 100, seed=3, step=0)
    assert ei.value.code == q2d.Q2D_ECAPACITY
    _, pos3, q3 = inputs(30000, np.float32, torch.float32)
    a = plan.rbm_step_noalloc(pos3, q3, 100, seed=3, step=1)
    r = plan.rbm_step(pos3, q3, 100, seed=3, step=1)
    torch.cuda.synchronize()
    same(a, r)
    # P above p_max: the same capacity error as the allocating call
    with pytest.raises(q2d.Q2DError) as ei:
        plan.rbm_step_noalloc(pos3, q3, 101, seed=3, step=1)
    assert ei.value.code == q2d.Q2D_ECAPACITY
    plan.close()
