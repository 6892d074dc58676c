"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars: FP64 results within 1e-10 relative (norm over all particles) of the
FP64 oracle on the same SOE table and modes; FP32 results within 1e-5 at these
sizes (1e-4 is the stated bar for the FP32 force at N = 1e6); sampled modes and
the sort's integer work bit-exact.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from _parity import assert_close, assert_energy  # noqa: E402

torch = pytest.importorskip("torch")

import paper_2403_01521_amd as q2d  # noqa: E402
import workloads as wl  # noqa: E402
from oracle import lattice, rbsampler, soewald2d  # noqa: E402
from oracle import recursion as o3  # noqa: E402


def dev(a, dt):
    return torch.tensor(np.asarray(a), dtype=dt, device="cuda")


def rel(a, b):
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def run_exact(c, w, s, prec, pos=None, q=None):
    dt = torch.float32 if prec == "fp32" else torch.float64
    pos = c["pos"] if pos is None else pos
    q = c["q"] if q is None else q
    plan = q2d.Plan(c["box"], c["alpha"], w, s, kc=c["kc"], precision=prec, n_max=max(1, len(q)))
    phi, F, E = plan.long_range(dev(pos, dt), dev(q, dt))
    torch.cuda.synchronize()
    out = phi.cpu().numpy().astype(np.float64), F.cpu().numpy().astype(np.float64), float(E.cpu()[0])
    plan.close()
    return out


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_exact_k_config1(soe_tables, prec, tol):
    c = wl.make_config(1, dtype=np.float32 if prec == "fp32" else np.float64)
    w, s = soe_tables[16]
    phi, F, E = run_exact(c, w, s, prec)
    r = soewald2d.exact_k(c["pos"], c["q"], c["box"], c["alpha"], c["kc"], w, s)
    print("config1", prec, rel(phi, r["phi"]), rel(F, r["F"]), abs(E - r["U"]) / abs(r["U"]))
    assert_close(phi, r["phi"], tol)
    assert_close(F, r["F"], tol)
    assert abs(E - r["U"]) < tol * abs(r["U"])


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-5)])
def test_exact_k_config2(soe_tables, prec, tol):
    c = wl.make_config(2, dtype=np.float32 if prec == "fp32" else np.float64)
    w, s = soe_tables[24]
    phi, F, E = run_exact(c, w, s, prec)
    m, wt = soewald2d.exact_modes(c["box"][0], c["box"][1], c["alpha"], c["kc"])
    r = o3.long_range(c["pos"], c["q"], c["box"], c["alpha"], w, s, m, wt, nthreads=8)
    print("config2", prec, len(m), rel(phi, r["phi"]), rel(F, r["F"]), abs(E - r["U"]) / abs(r["U"]))
    assert_close(phi, r["phi"], tol)
    assert_close(F, r["F"], tol)
    assert abs(E - r["U"]) < tol * abs(r["U"])
    # direct pair sums on sampled targets
    tg = np.random.default_rng(0).choice(len(c["q"]), 8, replace=False)
    r2 = soewald2d.exact_k(c["pos"], c["q"], c["box"], c["alpha"], c["kc"], w, s, targets=tg)
    assert_close(phi[tg], r2["phi"], tol)
    assert_close(F[tg], r2["F"], tol)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_rbm_step_matches_oracle(soe_tables, prec, tol):
    dtn = np.float32 if prec == "fp32" else np.float64
    dt = torch.float32 if prec == "fp32" else torch.float64
    c = wl.make_config(3, dtype=dtn, n_override=20000)
    w, s = soe_tables[16]
    box, alpha = c["box"], c["alpha"]
    P = 100
    plan = q2d.Plan(box, alpha, w, s, precision=prec, n_max=len(c["q"]), p_max=P)
    phi, F, E, modes = plan.rbm_step(dev(c["pos"], dt), dev(c["q"], dt), P, seed=7, step=3)
    torch.cuda.synchronize()
    phi = phi.cpu().numpy().astype(np.float64)
    F = F.cpu().numpy().astype(np.float64)
    E = float(E.cpu()[0])
    modes = modes.cpu().numpy()
    ref_modes, _ = rbsampler.sample_modes(7, 3, P, alpha, box[0], box[1])
    assert np.array_equal(modes, ref_modes)
    info = plan.info()
    H = lattice.H_direct(box[0], box[1], alpha)
    assert abs(info["H"] - H) < 1e-12 * H
    D = soewald2d.diag_constant(box[0], box[1], alpha, w, s)
    assert abs(info["diag_rb"] - D) < 1e-12 * abs(D)
    r = o3.long_range(c["pos"], c["q"], box, alpha, w, s, modes,
                      soewald2d.rb_weights(P, H, box[0], box[1]), include_self_pair=False,
                      diag=D, nthreads=8)
    print("rbm", prec, rel(phi, r["phi"]), rel(F, r["F"]), abs(E - r["U"]) / abs(r["U"]))
    assert_close(phi, r["phi"], tol)
    assert_close(F, r["F"], tol)
    assert abs(E - r["U"]) < tol * abs(r["U"])
    plan.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_rbm_step_reduced_soe(soe_tables, prec, tol):
    """The random-batch step with the model-reduced M = 10 SOE table (five
    conjugate pairs: other kernel instantiations than M = 16) against O3."""
    dtn = np.float32 if prec == "fp32" else np.float64
    dt = torch.float32 if prec == "fp32" else torch.float64
    c = wl.make_config(3, dtype=dtn, n_override=20000)
    w, s = soe_tables["r10"]
    box, alpha = c["box"], c["alpha"]
    P = 100
    plan = q2d.Plan(box, alpha, w, s, precision=prec, n_max=len(c["q"]), p_max=P)
    phi, F, E, modes = plan.rbm_step(dev(c["pos"], dt), dev(c["q"], dt), P, seed=8, step=5)
    torch.cuda.synchronize()
    modes = modes.cpu().numpy()
    H = lattice.H_direct(box[0], box[1], alpha)
    D = soewald2d.diag_constant(box[0], box[1], alpha, w, s)
    assert abs(plan.info()["diag_rb"] - D) < 1e-12 * abs(D)
    r = o3.long_range(c["pos"], c["q"], box, alpha, w, s, modes,
                      soewald2d.rb_weights(P, H, box[0], box[1]), include_self_pair=False,
                      diag=D, nthreads=8)
    phi = phi.cpu().numpy().astype(np.float64)
    F = F.cpu().numpy().astype(np.float64)
    print("rbm reduced SOE", prec, rel(phi, r["phi"]), rel(F, r["F"]))
    assert_close(phi, r["phi"], tol)
    assert_close(F, r["F"], tol)
    assert abs(float(E.cpu()[0]) - r["U"]) < tol * abs(r["U"])
    plan.close()


def test_empty_and_single(soe_tables):
    w, s = soe_tables[16]
    box = (10.0, 10.0, 4.0)
    plan = q2d.Plan(box, 0.5, w, s, kc=3.0, precision="fp64", n_max=8, p_max=4)
    pos = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    q = torch.zeros(0, dtype=torch.float64, device="cuda")
    phi, F, E = plan.long_range(pos, q)
    assert float(E.cpu()[0]) == 0.0
    phi, F, E, m = plan.rbm_step(pos, q, 4, 1, 1)
    assert float(E.cpu()[0]) == 0.0
    # one neutral "particle" (q = 0): everything vanishes
    p1 = torch.tensor([[1.0, 2.0, 3.0]], dtype=torch.float64, device="cuda")
    q1 = torch.zeros(1, dtype=torch.float64, device="cuda")
    phi, F, E = plan.long_range(p1, q1)
    assert float(phi.abs().max()) == 0.0 and float(F.abs().max()) == 0.0
    with pytest.raises(q2d.Q2DError):
        plan.long_range(torch.zeros((9, 3), dtype=torch.float64, device="cuda"),
                        torch.zeros(9, dtype=torch.float64, device="cuda"))
    with pytest.raises(q2d.Q2DError):
        plan.rbm_step(p1, q1, 5, 1, 1)
    plan.close()


@pytest.mark.parametrize("n", [2, 63, 64, 65, 1000, 4097])
def test_ragged_sizes_fp64(soe_tables, n):
    w, s = soe_tables[12]
    box = (12.0, 9.0, 3.0)
    pos, q = wl.random_system(n, box, seed=100 + n)
    c = dict(box=box, alpha=0.6, kc=3.5)
    phi, F, E = run_exact(c, w, s, "fp64", pos=pos, q=q)
    m, wt = soewald2d.exact_modes(box[0], box[1], 0.6, 3.5)
    r = o3.long_range(pos, q, box, 0.6, w, s, m, wt, nthreads=8)
    print("ragged", n, rel(phi, r["phi"]), rel(F, r["F"]))
    assert_close(phi, r["phi"], 1e-10)
    assert_close(F, r["F"], 1e-10)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_clustered_heights(soe_tables, prec, tol):
    """Heights packed into a layer 0.004 thick (9000 particles: one z bucket
    of the sort larger than its LDS capacity, sorted in global memory) and
    1500 at one height (ties: a bucket of equal keys), 500 more spread over
    the box.  Random batch step against the oracle on the same modes."""
    dtn = np.float32 if prec == "fp32" else np.float64
    dt = torch.float32 if prec == "fp32" else torch.float64
    rng = np.random.default_rng(4242)
    box, alpha, P = (40.0, 40.0, 10.0), 0.25, 32
    n_thin, n_tie, n_rest = 9000, 1500, 500
    n = n_thin + n_tie + n_rest
    z = np.concatenate([rng.uniform(2.0, 2.004, n_thin), np.full(n_tie, 7.5),
                        rng.uniform(0.0, 10.0, n_rest)])
    pos = np.stack([rng.uniform(0, box[0], n), rng.uniform(0, box[1], n), z], axis=1)
    q = rng.permutation(np.repeat([1.0, -1.0], n // 2))
    pos, q = pos.astype(dtn), q.astype(dtn)
    w, s = soe_tables[16]
    plan = q2d.Plan(box, alpha, w, s, precision=prec, n_max=n, p_max=P)
    phi, F, E, modes = plan.rbm_step(dev(pos, dt), dev(q, dt), P, seed=5, step=2)
    torch.cuda.synchronize()
    phi = phi.cpu().numpy().astype(np.float64)
    F = F.cpu().numpy().astype(np.float64)
    E = float(E.cpu()[0])
    modes = modes.cpu().numpy()
    H = lattice.H_direct(box[0], box[1], alpha)
    D = soewald2d.diag_constant(box[0], box[1], alpha, w, s)
    r = o3.long_range(pos, q, box, alpha, w, s, modes, soewald2d.rb_weights(P, H, box[0], box[1]),
                      include_self_pair=False, diag=D, nthreads=8)
    print("clustered", prec, rel(phi, r["phi"]), rel(F, r["F"]), abs(E - r["U"]) / abs(r["U"]))
    assert_close(phi, r["phi"], tol)
    assert_close(F, r["F"], tol)
    assert_energy(E, r["U"], q, r["phi"], tol)
    plan.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_sort_paths_agree(soe_tables, prec, monkeypatch):
    """The bucket sort (systems up to ~1.2e6 particles in FP32) and the radix
    sort (larger systems; Q2D_RADIX_SORT=1 forces it) realise the same
    (height, input index) order, so every output is bitwise the same; with
    ties and a dense layer on the bench workload's height profile."""
    dtn = np.float32 if prec == "fp32" else np.float64
    dt = torch.float32 if prec == "fp32" else torch.float64
    c = wl.make_config(3, dtype=dtn, n_override=200000)
    pos = c["pos"].copy()
    pos[:3000, 2] = 4.25
    pos[3000:9000, 2] = np.linspace(6.0, 6.001, 6000, dtype=dtn)
    w, s = soe_tables[16]
    plan = q2d.Plan(c["box"], c["alpha"], w, s, precision=prec, n_max=len(c["q"]), p_max=64)
    gp, gq = dev(pos, dt), dev(c["q"], dt)
    a = [t.clone() for t in plan.rbm_step(gp, gq, 64, seed=3, step=1)]
    monkeypatch.setenv("Q2D_RADIX_SORT", "1")
    b = [t.clone() for t in plan.rbm_step(gp, gq, 64, seed=3, step=1)]
    monkeypatch.delenv("Q2D_RADIX_SORT")
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    plan.close()


@pytest.mark.parametrize("sampler", ["metropolis", "iid"])
def test_modes_sampled_ahead(soe_tables, sampler):
    """A random-batch step samples the next step's modes on the internal
    stream; the next call on the same stream with (seed, step + 1, P) uses
    them.  Every such call, and every call that cannot use them (another step,
    another P, another stream, the allocation-free entry point in between),
    gives bitwise what a fresh plan gives for that (seed, step, P)."""
    c = wl.make_config(3, dtype=np.float32, n_override=30000)
    w, s = soe_tables[16]
    gp, gq = dev(c["pos"], torch.float32), dev(c["q"], torch.float32)

    def make():
        return q2d.Plan(c["box"], c["alpha"], w, s, precision="fp32", n_max=len(c["q"]),
                        p_max=96, sampler=sampler)

    def fresh(P, step):
        f = make()
        out = [x.clone() for x in f.rbm_step(gp, gq, P, seed=11, step=step)]
        f.close()
        return out

    plan = make()
    other = torch.cuda.Stream()
    calls = [(64, 5), (64, 6), (64, 7), (64, 9), (96, 10), (64, 11), (64, 12), ("noalloc", 13),
             (64, 13), ("stream", 14), (64, 15)]
    for P, step in calls:
        if P == "noalloc":
            got = [x.clone() for x in plan.rbm_step_noalloc(gp, gq, 64, seed=11, step=step)]
            P = 64
        elif P == "stream":
            P = 64
            other.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(other):
                got = [x.clone() for x in plan.rbm_step(gp, gq, P, seed=11, step=step)]
            torch.cuda.current_stream().wait_stream(other)
        else:
            got = [x.clone() for x in plan.rbm_step(gp, gq, P, seed=11, step=step)]
        ref = fresh(P, step)
        for x, y in zip(got, ref):
            assert torch.equal(x, y), (P, step)
    assert plan.check() == 0
    plan.close()


@pytest.mark.parametrize("entry", ["rbm_step", "rbm_step_noalloc"])
def test_step_captured_by_caller(soe_tables, entry):
    """A caller captures one random-batch step into a graph (scratch already
    allocated by an eager call): every replay, with eager steps of other draws
    and synchronisations in between, gives bitwise the eager result of the
    captured (seed, step), and the eager steps around the replays (consecutive
    draws, which would use modes sampled ahead) give bitwise what a fresh plan
    gives: a replay rewrites the plan's mode buffers."""
    c = wl.make_config(3, dtype=np.float32, n_override=20000)
    w, s = soe_tables[16]
    gp, gq = dev(c["pos"], torch.float32), dev(c["q"], torch.float32)
    P = 64
    plan = q2d.Plan(c["box"], c["alpha"], w, s, precision="fp32", n_max=len(c["q"]), p_max=P)
    step = getattr(plan, entry)
    ref = [x.clone() for x in plan.rbm_step(gp, gq, P, seed=21, step=7)]
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        step(gp, gq, P, seed=21, step=6)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(cs)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cs):
        out = step(gp, gq, P, seed=21, step=7)
    torch.cuda.synchronize()
    def fresh(st):
        f = q2d.Plan(c["box"], c["alpha"], w, s, precision="fp32", n_max=len(c["q"]), p_max=P)
        o = [x.clone() for x in f.rbm_step(gp, gq, P, seed=21, step=st)]
        f.close()
        return o

    def eager(st):
        got = [x.clone() for x in plan.rbm_step(gp, gq, P, seed=21, step=st)]
        for x, y in zip(got, fresh(st)):
            assert torch.equal(x, y), (entry, st)

    # consecutive eager steps with replays between them (steps 8, 9, replay,
    # 10, 11, replay, ...): with modes sampled ahead, one of the replays would
    # land on the buffer that holds the next step's modes
    st = 8
    for r in range(3):
        eager(st)
        eager(st + 1)
        g.replay()
        torch.cuda.synchronize()
        for x, y in zip(out, ref):
            assert torch.equal(x, y), (entry, r)
        st += 2
    eager(st)
    assert plan.check() == 0
    del g
    plan.close()


def test_equal_heights_square_lattice(soe_tables):
    """All ions in one plane (sort ties): the square ionic lattice."""
    w, s = soe_tables[24]
    a = 1.0
    cell, qc = wl.square_ionic_cell(a, 0.5)
    # 8 x 8 copies of the cell in a 16 x 16 box
    pos = np.concatenate([cell + [2 * a * i, 2 * a * j, 0] for i in range(8) for j in range(8)])
    q = np.tile(qc, 64)
    box = (16.0, 16.0, 1.0)
    c = dict(box=box, alpha=1.2, kc=1.2 * 12)
    phi, F, E = run_exact(c, w, s, "fp64", pos=pos, q=q)
    r = soewald2d.exact_k(pos, q, box, 1.2, 1.2 * 12, w, s, targets=np.arange(4))
    assert_close(phi[:4], r["phi"], 1e-10)
    assert np.abs(F).max() < 1e-9


def test_deterministic(soe_tables):
    w, s = soe_tables[16]
    c = wl.make_config(3, dtype=np.float32, n_override=30000)
    plan = q2d.Plan(c["box"], c["alpha"], w, s, precision="fp32", n_max=30000, p_max=100)
    pos, q = dev(c["pos"], torch.float32), dev(c["q"], torch.float32)
    a = [t.clone() for t in plan.rbm_step(pos, q, 100, 5, 9)]
    b = [t.clone() for t in plan.rbm_step(pos, q, 100, 5, 9)]
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    plan.close()


def test_kernel_timers_and_stride(soe_tables):
    """The measurement hooks: with timers on every call each family records one
    launch per step (the sweep is one launch per step); with stride n only every
    n-th call records, and results do not depend on either."""
    c = wl.make_config(3, dtype=np.float32, n_override=20000)
    w, s = soe_tables[16]
    P = 100
    plan = q2d.Plan(c["box"], c["alpha"], w, s, precision="fp32", n_max=len(c["q"]), p_max=P)
    pos, q = dev(c["pos"], torch.float32), dev(c["q"], torch.float32)
    ref = plan.rbm_step(pos, q, P, seed=3, step=1)[1].cpu().numpy()
    plan.timing_enable(1 << q2d.TIMER_SWEEP | 1 << q2d.TIMER_CALL)
    for k in range(8):
        plan.rbm_step(pos, q, P, seed=3, step=1)
    ms, cnt = plan.timing_read(q2d.TIMER_SWEEP)
    assert cnt == 8 and ms > 0
    assert plan.timing_read(q2d.TIMER_CALL)[1] == 8
    plan.timing_enable(1 << q2d.TIMER_SWEEP)
    plan.timing_stride(4)
    for k in range(8):
        F = plan.rbm_step(pos, q, P, seed=3, step=1)[1]
    assert plan.timing_read(q2d.TIMER_SWEEP)[1] == 2
    assert np.array_equal(F.cpu().numpy(), ref)
    with pytest.raises(q2d.Q2DError):
        plan.timing_stride(0)
    plan.close()
