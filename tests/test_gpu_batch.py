"""Replica batches (q2d_batch_*): R systems of uneven size in one step.

* every replica equals the single-system q2d_rbm_step for its box and derived
  seed (modes bit-exact; FP64 within 1e-12, FP32 within 1e-5), including empty
  and one-particle replicas and boxes with Lx != Ly;
* one replica against the oracle (O3 with the oracle's own H and j = i
  constant for that box), FP64 within 1e-10, and two replicas of an FP32
  batch against O3 directly within 1e-5;
* results independent of the segment length (64 ... 512) and of the other
  launch shapes (sweep work-group split, aggregate chunks per wave);
* a captured step replayed as a hipGraph equals the eager steps it stands
  for, replay after replay (the step number advances on the device);
* the tuner returns one of the candidates, leaves results unchanged, and a
  second tune of the same shape reuses the cached choice;
* configuration 5 at full size (256 replicas, 1.65e6 particles, P = 64):
  four replicas against single-system plans.
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

ALPHA = 0.3
P = 64


def dev(a, dt):
    return torch.tensor(np.asarray(a), dtype=dt, device="cuda")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def small_batch(dtype):
    rng = np.random.Generator(np.random.PCG64(5005))
    counts = np.array([0, 1, 64, 700, 2500, 4098, 257], dtype=np.int64)
    boxes = np.array([[30, 30, 6], [12, 20, 4], [20, 20, 6], [40, 35, 6], [60, 60, 6],
                      [80, 70, 5], [25, 25, 6]], dtype=np.float64)
    pos, q = [], []
    for n, b in zip(counts, boxes):
        p, qq = wl.uniform_ions(rng, n // 2, n - n // 2, tuple(b))
        pos.append(p.reshape(-1, 3))
        q.append(qq)
    return (np.concatenate(pos).astype(dtype), np.concatenate(q).astype(dtype), boxes, counts)


def single(box, pos, q, w, s, prec, seed, step):
    dt = torch.float32 if prec == "fp32" else torch.float64
    plan = q2d.Plan(box, ALPHA, w, s, precision=prec, n_max=max(len(q), 1), p_max=P)
    phi, F, E, m = plan.rbm_step(dev(pos, dt), dev(q, dt), P, seed, step)
    torch.cuda.synchronize()
    out = (phi.double().cpu().numpy(), F.double().cpu().numpy(), float(E.cpu()[0]),
           m.cpu().numpy())
    plan.close()
    return out


def run_batch(b, pos, q, dt, seed, step):
    phi, F, E, m = b.rbm_step(dev(pos, dt), dev(q, dt), P, seed, step)
    torch.cuda.synchronize()
    return (phi.double().cpu().numpy(), F.double().cpu().numpy(), E.cpu().numpy(),
            m.cpu().numpy())


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_batch_matches_single_plans(soe_tables, prec, tol):
    dtn = np.float32 if prec == "fp32" else np.float64
    dt = torch.float32 if prec == "fp32" else torch.float64
    pos, q, boxes, counts = small_batch(dtn)
    w, s = soe_tables[16]
    b = q2d.Batch(boxes, counts, ALPHA, w, s, precision=prec, p_max=P)
    seed, step = 123, 7
    phi, F, E, modes = run_batch(b, pos, q, dt, seed, step)
    off = np.concatenate([[0], np.cumsum(counts)])
    for r in range(len(counts)):
        sl = slice(off[r], off[r + 1])
        ph1, F1, E1, m1 = single(boxes[r], pos[sl], q[sl], w, s, prec, q2d.replica_seed(seed, r),
                                 step)
        assert np.array_equal(modes[r], m1), r
        if counts[r] == 0:
            assert E[r] == 0.0
            continue
        assert_close(phi[sl], ph1, tol, r)
        assert_close(F[sl], F1, tol, r)
        assert abs(E[r] - E1) <= tol * abs(E1), (r, E[r], E1)
    b.close()


def test_batch_replica_vs_oracle(soe_tables):
    pos, q, boxes, counts = small_batch(np.float64)
    w, s = soe_tables[16]
    b = q2d.Batch(boxes, counts, ALPHA, w, s, precision="fp64", p_max=P)
    phi, F, E, modes = run_batch(b, pos, q, torch.float64, 9, 2)
    off = np.concatenate([[0], np.cumsum(counts)])
    r = 5
    sl = slice(off[r], off[r + 1])
    box = boxes[r]
    H = lattice.H_direct(box[0], box[1], ALPHA)
    D = soewald2d.diag_constant(box[0], box[1], ALPHA, w, s)
    info = b.info()
    assert abs(info["H"][r] - H) < 1e-12 * H
    assert abs(info["diag_rb"][r] - D) < 1e-10 * abs(D)
    ref = o3.long_range(pos[sl], q[sl], box, ALPHA, w, s, modes[r],
                        soewald2d.rb_weights(P, H, box[0], box[1]), include_self_pair=False,
                        diag=D, nthreads=8)
    assert_close(phi[sl], ref["phi"], 1e-10)
    assert_close(F[sl], ref["F"], 1e-10)
    assert abs(E[r] - ref["U"]) < 1e-10 * abs(ref["U"])
    b.close()


def test_batch_fp32_replicas_vs_oracle(soe_tables):
    """Two replicas of an FP32 batch (a 700- and a 4098-particle box) against
    O3 in FP64 on the same modes, each with the oracle's own H and j = i
    constant for its box."""
    pos, q, boxes, counts = small_batch(np.float32)
    w, s = soe_tables[16]
    b = q2d.Batch(boxes, counts, ALPHA, w, s, precision="fp32", p_max=P)
    phi, F, E, modes = run_batch(b, pos, q, torch.float32, 21, 6)
    off = np.concatenate([[0], np.cumsum(counts)])
    for r in (3, 5):
        sl = slice(off[r], off[r + 1])
        box = boxes[r]
        H = lattice.H_direct(box[0], box[1], ALPHA)
        D = soewald2d.diag_constant(box[0], box[1], ALPHA, w, s)
        ref = o3.long_range(pos[sl].astype(np.float64), q[sl].astype(np.float64), box, ALPHA,
                            w, s, modes[r], soewald2d.rb_weights(P, H, box[0], box[1]),
                            include_self_pair=False, diag=D, nthreads=8)
        print("fp32 replica %d: F %.2e phi %.2e" % (r, rel(F[sl], ref["F"]),
                                                    rel(phi[sl], ref["phi"])))
        assert_close(phi[sl], ref["phi"], 1e-5)
        assert_close(F[sl], ref["F"], 1e-5)
        assert abs(E[r] - ref["U"]) < 1e-5 * abs(ref["U"])
    b.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_batch_launch_shape_invariance(soe_tables, prec, tol):
    """Every launch shape the tuner may pick gives the same results to
    rounding (the segment length, the sweep's split, the aggregate pass's
    chunks per wave): FP64 against the default shape within 1e-12; FP32, whose
    segmentations round differently, each against the FP64 result within 2e-5
    (the FP32 rounding bound of a 512-step segment with the SOE weights'
    cancellation is about 3e-5; observed up to 1.1e-5 on these mixed small
    replicas)."""
    dtn = np.float32 if prec == "fp32" else np.float64
    dt = torch.float32 if prec == "fp32" else torch.float64
    pos, q, boxes, counts = small_batch(dtn)
    w, s = soe_tables[16]
    b = q2d.Batch(boxes, counts, ALPHA, w, s, precision=prec, p_max=P)
    assert b.config() == {"segment": 256, "split": 1, "agg_cpw": 2}
    if prec == "fp64":
        ref = run_batch(b, pos, q, dt, 4, 2)
    else:
        b64 = q2d.Batch(boxes, counts, ALPHA, w, s, precision="fp64", p_max=P)
        ref = run_batch(b64, pos.astype(np.float64), q.astype(np.float64), torch.float64, 4, 2)
        b64.close()
    for S, split, cpw in ((256, 2, 1), (128, 1, 4), (512, 2, 2), (64, 1, 1)):
        b.set_config(S, split, cpw)
        assert b.config() == {"segment": S, "split": split, "agg_cpw": cpw}
        out = run_batch(b, pos, q, dt, 4, 2)
        assert np.array_equal(out[3], ref[3])
        print(prec, (S, split, cpw), "phi %.2e F %.2e" % (rel(out[0], ref[0]), rel(out[1], ref[1])))
        assert_close(out[0], ref[0], tol, (S, split, cpw))
        assert_close(out[1], ref[1], tol, (S, split, cpw))
    for bad in ((100, 1, 2), (256, 3, 2), (256, 1, 3)):
        with pytest.raises(q2d.Q2DError) as ei:
            b.set_config(*bad)
        assert ei.value.code == q2d.Q2D_EINVAL
    b.close()


def test_batch_segment_length_invariance(soe_tables):
    pos, q, boxes, counts = small_batch(np.float64)
    w, s = soe_tables[16]
    b = q2d.Batch(boxes, counts, ALPHA, w, s, precision="fp64", p_max=P)
    ref = run_batch(b, pos, q, torch.float64, 3, 1)
    for S in (64, 128, 512):
        b.set_segment(S)
        assert b.info()["segment"] == S
        out = run_batch(b, pos, q, torch.float64, 3, 1)
        assert np.array_equal(out[3], ref[3])
        assert_close(out[0], ref[0], 1e-12)
        assert_close(out[1], ref[1], 1e-12)
        assert np.allclose(out[2], ref[2], rtol=1e-12, atol=0)
    b.close()


def test_batch_graph_replay_matches_eager(soe_tables):
    pos, q, boxes, counts = small_batch(np.float32)
    w, s = soe_tables[16]
    seed, step0 = 77, 5
    eager = q2d.Batch(boxes, counts, ALPHA, w, s, precision="fp32", p_max=P)
    graph = q2d.Batch(boxes, counts, ALPHA, w, s, precision="fp32", p_max=P)
    gp, gq = dev(pos, torch.float32), dev(q, torch.float32)
    phi_g, F_g, E_g = graph.capture(gp, gq, P, seed, step0)
    for k in range(3):
        graph.replay(1)
        torch.cuda.synchronize()
        got = (phi_g.cpu().numpy().copy(), F_g.cpu().numpy().copy(), E_g.cpu().numpy().copy())
        ref = run_batch(eager, pos, q, torch.float32, seed, step0 + k)
        assert np.array_equal(got[0], ref[0].astype(np.float32)), k
        assert np.array_equal(got[1], ref[1].astype(np.float32)), k
        assert np.array_equal(got[2], ref[2]), k
    # several replays in one call advance the step as many times
    graph.replay(2)
    torch.cuda.synchronize()
    ref = run_batch(eager, pos, q, torch.float32, seed, step0 + 4)
    assert np.array_equal(phi_g.cpu().numpy(), ref[0].astype(np.float32))
    eager.close()
    graph.close()


def test_batch_graph_dropped_when_scratch_grows(soe_tables):
    """A graph holds the addresses of the scratch it was captured with.  An
    eager step with a larger P grows the mode tables and aggregates; replay
    must then refuse (Q2D_EUNSUPPORTED) or, if nothing moved, replay exactly
    the captured step.  A new capture afterwards works again."""
    pos, q, boxes, counts = small_batch(np.float32)
    w, s = soe_tables[16]
    seed, step0 = 31, 2
    b = q2d.Batch(boxes, counts, ALPHA, w, s, precision="fp32", p_max=P)
    ref_b = q2d.Batch(boxes, counts, ALPHA, w, s, precision="fp32", p_max=P)
    gp, gq = dev(pos, torch.float32), dev(q, torch.float32)
    phi_g, F_g, E_g = b.capture(gp, gq, 32, seed, step0)
    b.rbm_step(gp, gq, P, seed, step0 + 100)
    torch.cuda.synchronize()
    try:
        b.replay(1)
    except q2d.Q2DError as e:
        assert e.code == q2d.Q2D_EUNSUPPORTED, e
    else:
        torch.cuda.synchronize()
        ref = ref_b.rbm_step(gp, gq, 32, seed, step0)
        torch.cuda.synchronize()
        assert torch.equal(phi_g, ref[0]) and torch.equal(F_g, ref[1])
    phi_g, F_g, E_g = b.capture(gp, gq, P, seed, step0)
    b.replay(1)
    torch.cuda.synchronize()
    ref = ref_b.rbm_step(gp, gq, P, seed, step0)
    torch.cuda.synchronize()
    assert torch.equal(phi_g, ref[0]) and torch.equal(F_g, ref[1]) and torch.equal(E_g, ref[2])
    b.close()
    ref_b.close()


def test_batch_tune(soe_tables):
    pos, q, boxes, counts = small_batch(np.float32)
    w, s = soe_tables[16]
    b = q2d.Batch(boxes, counts, ALPHA, w, s, precision="fp32", p_max=P)
    ref = run_batch(b, pos, q, torch.float32, 1, 1)
    S = b.tune(dev(pos, torch.float32), dev(q, torch.float32), P, seed=1)
    cfg = b.config()
    assert S in (64, 128, 256, 512) and b.info()["segment"] == S == cfg["segment"]
    assert cfg["split"] in (1, 2) and cfg["agg_cpw"] in (1, 2, 4)
    out = run_batch(b, pos, q, torch.float32, 1, 1)
    assert np.array_equal(out[3], ref[3])
    assert_close(out[1], ref[1], 1e-5)
    b.close()
    # a new batch of the same shape: the tune applies the cached choice
    b2 = q2d.Batch(boxes, counts, ALPHA, w, s, precision="fp32", p_max=P)
    b2.set_config(64, 2, 4 if cfg["agg_cpw"] != 4 else 1)
    assert b2.tune(dev(pos, torch.float32), dev(q, torch.float32), P, seed=1) == S
    assert b2.config() == cfg
    b2.close()


def test_batch_config5_fullsize(soe_tables):
    c = wl.make_replicas(dtype=np.float32)
    w, s = soe_tables[16]
    counts, boxes = c["counts"], c["boxes"]
    b = q2d.Batch(boxes, counts, c["alpha"], w, s, precision="fp32", p_max=c["P"])
    phi, F, E, modes = run_batch(b, c["pos"], c["q"], torch.float32, 11, 4)
    assert np.all(np.isfinite(phi)) and np.all(np.isfinite(F)) and np.all(np.isfinite(E))
    off = np.concatenate([[0], np.cumsum(counts)])
    picks = [int(np.argmin(counts)), int(np.argmax(counts)), 17, 200]
    for r in picks:
        sl = slice(off[r], off[r + 1])
        ph1, F1, E1, m1 = single(boxes[r], c["pos"][sl], c["q"][sl], w, s, "fp32",
                                 q2d.replica_seed(11, r), 4)
        assert np.array_equal(modes[r], m1)
        print("config5 replica %d (N=%d): F %.2e phi %.2e" % (r, counts[r], rel(F[sl], F1),
                                                             rel(phi[sl], ph1)))
        assert_close(F[sl], F1, 1e-5)
        assert_close(phi[sl], ph1, 1e-5)
    b.close()
