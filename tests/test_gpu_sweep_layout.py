"""The sweep's work-group layouts give the same results.

By default every k != 0 sweep work-group runs one direction (forward or
backward) of one unit block and writes its own output chunk.
Q2D_SPLIT=0 runs both directions in one work-group, the backward pass adding
to the forward pass's chunk.  Both layouts must agree with the FP64 oracle
(FP64 within 1e-10), and with each other up to the order of the final sums
(FP64 1e-13, FP32 2e-6 relative).  The mode counts cover full 64-mode groups
and every band width: P = 100 is 64 + 32 + 4 (F = 1, 2, 16), P = 37 is
32 + 8 (F = 2, 8; three padded lanes), P = 200 is 3 x 64 + 8.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from _parity import assert_close  # noqa: E402

torch = pytest.importorskip("torch")

import paper_2403_01521_amd as q2d  # noqa: E402
import workloads as wl  # noqa: E402
from oracle import lattice, soewald2d  # noqa: E402
from oracle import recursion as o3  # noqa: E402


def rel(a, b):
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / np.linalg.norm(b))


def step(c, w, s, prec, P, split, monkeypatch):
    dt = torch.float32 if prec == "fp32" else torch.float64
    monkeypatch.setenv("Q2D_SPLIT", "1" if split else "0")
    plan = q2d.Plan(c["box"], c["alpha"], w, s, precision=prec, n_max=len(c["q"]), p_max=P)
    phi, F, E, modes = plan.rbm_step(torch.tensor(c["pos"], device="cuda"),
                                     torch.tensor(c["q"], device="cuda"), P, seed=11, step=5)
    torch.cuda.synchronize()
    out = (phi.cpu().numpy().astype(np.float64), F.cpu().numpy().astype(np.float64),
           float(E.cpu()[0]), modes.cpu().numpy())
    plan.close()
    monkeypatch.delenv("Q2D_SPLIT")
    return out


@pytest.mark.parametrize("P", [100, 37, 200])
def test_split_layouts_fp64_vs_oracle(soe_tables, P, monkeypatch):
    c = wl.make_config(3, dtype=np.float64, n_override=6000)
    w, s = soe_tables[16]
    box, alpha = c["box"], c["alpha"]
    a = step(c, w, s, "fp64", P, True, monkeypatch)
    b = step(c, w, s, "fp64", P, False, monkeypatch)
    assert np.array_equal(a[3], b[3])
    H = lattice.H_direct(box[0], box[1], alpha)
    D = soewald2d.diag_constant(box[0], box[1], alpha, w, s)
    r = o3.long_range(c["pos"], c["q"], box, alpha, w, s, a[3],
                      soewald2d.rb_weights(P, H, box[0], box[1]), include_self_pair=False,
                      diag=D, nthreads=8)
    for out in (a, b):
        assert_close(out[0], r["phi"], 1e-10)
        assert_close(out[1], r["F"], 1e-10)
        assert abs(out[2] - r["U"]) < 1e-10 * abs(r["U"])
    assert_close(a[0], b[0], 1e-13)
    assert_close(a[1], b[1], 1e-13)


@pytest.mark.parametrize("P", [100, 37])
def test_split_layouts_fp32_agree(soe_tables, P, monkeypatch):
    c = wl.make_config(3, dtype=np.float32, n_override=20000)
    w, s = soe_tables[16]
    a = step(c, w, s, "fp32", P, True, monkeypatch)
    b = step(c, w, s, "fp32", P, False, monkeypatch)
    assert np.array_equal(a[3], b[3])
    print("fp32 split vs joint", P, rel(a[0], b[0]), rel(a[1], b[1]))
    assert_close(a[0], b[0], 2e-6)
    assert_close(a[1], b[1], 2e-6)
    assert abs(a[2] - b[2]) < 2e-6 * abs(b[2])
