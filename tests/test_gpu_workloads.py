"""GPU parity at the benchmark's full sizes and on the batched serving path.

* RGB-D 30k (the benchmark workload): full F, omega, v against the oracle at
  poses of the GPU trajectory, in the launch configuration bench.py times.
* Dense 300k: per-target terms of sampled targets against the oracle (each
  sampled target's sum over all sources), with the cutoff and by brute force;
  properties that hold at any size (swap symmetry, determinism).
* Batched submit/poll: every request's result equals the synchronous path's
  bitwise, alone and mixed with other requests; error paths.
Tolerances as in test_gpu_parity (reading C12): 1e-5 relative on F,
1e-5 of sum|terms| on omega and v; per-target F_j 2e-5.
"""
import numpy as np
import pytest

import oracle
from paper_1904_02266_amd import (CVO_ENOMEM, CVO_ENOOVERLAP, CVO_ENOTFOUND, CVO_EINVAL, Context, CvoError, Params,
                                  params_planes, params_rgbd, synth)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def check(g, ref, rtol=1e-5, what=""):
    r, A = ref["g"], ref["abs"]
    assert abs(g[0] - r[0]) <= rtol * r[0], (what, "F", g[0], r[0])
    for k in range(1, 7):
        assert abs(g[k] - r[k]) <= rtol * A[k], (what, k, g[k], r[k], (g[k] - r[k]) / A[k])


@pytest.fixture(scope="module")
def rgbd30k():
    return synth.rgbd_pair(30000, 30000, seed=2)


@pytest.fixture(scope="module")
def dense300k():
    return synth.rgbd_pair(300000, 300000, seed=3, select="random")


def test_rgbd30k_full_eval_along_trajectory(ctx, rgbd30k):
    import torch
    p = rgbd30k
    dev = torch.device("cuda:0")
    t = [torch.from_numpy(a).to(dev) for a in (p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat)]
    prm = params_rgbd(trace=True)
    out = ctx.register(*t, prm)
    tr = ctx.trace()
    assert out["iters"] == 100 and tr.shape[0] == 100
    a2 = oracle.mean_sqnorm(p.src_xyz)
    for k in (0, 30, 60, 99):
        Tk = np.eye(4) if k == 0 else tr[k - 1, 10:26].reshape(4, 4)
        ref = oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, Tk, ell=tr[k, 8], kappa=3.0, a2=a2)
        check(tr[k, :7], ref, what=f"iter {k}")
        assert abs(tr[k, 9] - ref["within"]) <= 1e-6 * ref["within"] + 50


def test_dense300k_sampled_targets_cutoff(ctx, dense300k):
    p = dense300k
    T = p.T_true
    prm = Params(stage_ell=(0.05,), cutoff_mult=3.0)
    sel = np.random.default_rng(7).choice(p.tgt_xyz.shape[0], 48, replace=False).astype(np.int32)
    out = ctx.eval_targets(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, prm, sel=sel)
    ref = oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, ell=0.05, kappa=3.0, sel=sel,
                      per_target=True)["per_target"]
    nz = ref[:, 0] > 0
    assert nz.sum() > 40
    np.testing.assert_allclose(out[nz, 0], ref[nz, 0], rtol=2e-5)
    # the gradient terms of a target: error against the target's own magnitude
    scale = np.abs(ref[:, 1:]).max(axis=1, keepdims=True) + 1e-300
    assert (np.abs(out[:, 1:] - ref[:, 1:]) <= 2e-5 * scale + 1e-12).all()


def test_dense300k_sampled_targets_brute_force(ctx, dense300k):
    p = dense300k
    T = p.T_true
    prm = Params(stage_ell=(0.1,), cutoff_mult=0.0)
    sel = np.random.default_rng(8).choice(p.tgt_xyz.shape[0], 16, replace=False).astype(np.int32)
    out = ctx.eval_targets(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, prm, sel=sel)
    ref = oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, ell=0.1, kappa=0.0, sel=sel,
                      per_target=True)["per_target"]
    np.testing.assert_allclose(out[:, 0], ref[:, 0], rtol=2e-5)


def test_dense300k_swap_symmetry_and_determinism(ctx, dense300k):
    """F(T; X, Z) = F(T^-1; Z, X) at full size (the oracle cannot afford the
    9e10-pair brute-force sum; the property holds at any size)."""
    p = dense300k
    T = p.T_true
    for ell in (0.2, 0.08, 0.05):
        prm = Params(stage_ell=(ell,), cutoff_mult=3.0)
        a = ctx.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, prm)
        b = ctx.eval(p.tgt_xyz, p.tgt_feat, p.src_xyz, p.src_feat, synth.invert_rigid(T), prm)
        assert abs(a[0] - b[0]) <= 2e-5 * a[0], ell
    a2 = ctx.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, prm)
    assert np.array_equal(a, a2)


def _small_requests(k0, count):
    reqs = []
    for k in range(count):
        n = 3000 + 1700 * k
        m = 2500 + 1300 * ((k * 7) % count)
        reqs.append(synth.rgbd_pair(n, m, seed=6000 + k0 + k))
    return reqs


def test_batched_equals_sync_alone_and_mixed():
    prm = params_rgbd(max_iters=20, stage_iters=(5, 5, 5))
    reqs = _small_requests(0, 6)
    ctx = Context(0, max_slots=8)
    try:
        sync = [ctx.register(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm) for q in reqs]
        # alone: one request at a time through the scheduler
        alone = []
        for q in reqs:
            tk, keep = ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)
            alone.append(ctx.poll(tk))
        # mixed: all at once, plus unrelated traffic in between
        extra = _small_requests(100, 3)
        tks = []
        for i, q in enumerate(reqs):
            tks.append(ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)[0])
            if i < len(extra):
                e = extra[i]
                ctx.submit(e.src_xyz, e.src_feat, e.tgt_xyz, e.tgt_feat,
                           params_rgbd(max_iters=33, stage_iters=(3, 3, 3)))
        mixed = [ctx.poll(t) for t in tks]
    finally:
        ctx.close()
    for s, a, m in zip(sync, alone, mixed):
        assert a["rc"] == 0 and m["rc"] == 0
        assert a["iters"] == 20 and m["iters"] == 20
        assert np.array_equal(s["T"], a["T"]) and np.array_equal(a["T"], m["T"])
        assert s["F"] == a["F"] == m["F"]


def test_batched_graph_chunks_equal_direct_launches():
    """With cvo_set_graphs(1) the scheduler captures a chunk of iterations
    once per launch layout and replays it while the layout holds; the results
    equal the direct launches' and the synchronous ones bit for bit.  The
    batch runs twice (the second replays the graph cached from the first,
    with the scheduler's own copies and synchronisations between replays),
    and a mixed run with late arrivals under another step rule changes the
    layout (new captures)."""
    prm = params_rgbd(max_iters=20, stage_iters=(5, 5, 5))
    reqs = _small_requests(300, 6)
    ctx = Context(0, max_slots=8)
    try:
        sync = [ctx.register(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm) for q in reqs]
        direct = [ctx.poll(t) for t in [ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)[0]
                                        for q in reqs]]
        assert ctx.serving_stats()["graph_chunks"] == 0
        ctx.set_graphs(True)
        runs = []
        for _ in range(2):
            tks = [ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)[0] for q in reqs]
            runs.append([ctx.poll(t) for t in tks])
        replayed = ctx.serving_stats()["graph_chunks"]
        extra = _small_requests(400, 3)
        tks = []
        for i, q in enumerate(reqs):
            tks.append(ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)[0])
            if i < len(extra):
                e = extra[i]
                ctx.submit(e.src_xyz, e.src_feat, e.tgt_xyz, e.tgt_feat,
                           params_rgbd(max_iters=12, stage_iters=(3, 3, 3), step_rule="quartic"))
        runs.append([ctx.poll(t) for t in tks])
        ctx.set_graphs(False)
    finally:
        ctx.close()
    assert replayed >= 6, replayed      # three chunks per run of 20 iterations, two runs
    for k, s in enumerate(sync):
        assert direct[k]["rc"] == 0 and np.array_equal(s["T"], direct[k]["T"]) and s["F"] == direct[k]["F"]
        for run in runs:
            o = run[k]
            assert o["rc"] == 0 and o["iters"] == 20
            assert np.array_equal(s["T"], o["T"]) and s["F"] == o["F"], k


def test_concurrent_submitters_and_synchronous_calls():
    """cvo_submit and cvo_poll from four threads at once while the main
    thread makes synchronous cvo_register calls on the same context (they
    serialise on the context; the scheduler runs on its own stream): every
    result equals the synchronous one bit for bit."""
    import threading
    prm = params_rgbd(max_iters=12, stage_iters=(3, 3, 3))
    reqs = _small_requests(500, 16)
    ctx = Context(0, max_slots=32)
    results = [None] * len(reqs)
    errors = []
    try:
        sync = [ctx.register(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm) for q in reqs]

        def worker(ids):
            try:
                tks = [(i, ctx.submit(reqs[i].src_xyz, reqs[i].src_feat, reqs[i].tgt_xyz, reqs[i].tgt_feat,
                                      prm)[0]) for i in ids]
                for i, t in tks:
                    results[i] = ctx.poll(t)
            except Exception as e:  # reported below
                errors.append(e)

        threads = [threading.Thread(target=worker, args=(list(range(k, len(reqs), 4)),)) for k in range(4)]
        for t in threads:
            t.start()
        again = [ctx.register(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm) for q in reqs[:4]]
        for t in threads:
            t.join(timeout=120)
        assert not any(t.is_alive() for t in threads)
        stats = ctx.serving_stats()
    finally:
        ctx.close()
    assert not errors, errors
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    for s, o in zip(sync, results):
        assert o is not None and o["rc"] == 0 and o["iters"] == 12
        assert np.array_equal(s["T"], o["T"]) and s["F"] == o["F"]
    for s, a in zip(sync, again):
        assert np.array_equal(s["T"], a["T"]) and s["F"] == a["F"]


def test_destroy_with_outstanding_requests():
    """cvo_destroy waits for the requests still queued or running (their
    work is bounded by their iteration cap) and frees everything; a context
    created afterwards on the same device works."""
    import time
    prm = params_rgbd(max_iters=12, stage_iters=(3, 3, 3))
    reqs = _small_requests(600, 10)
    ctx = Context(0, max_slots=4)
    for q in reqs:
        ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)
    t0 = time.perf_counter()
    ctx.close()                                  # nothing polled
    assert time.perf_counter() - t0 < 60.0
    ctx = Context(0, max_slots=4)
    try:
        q = reqs[0]
        a = ctx.register(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)
        b = ctx.poll(ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)[0])
    finally:
        ctx.close()
    assert a["rc"] == 0 and b["rc"] == 0 and np.array_equal(a["T"], b["T"])


def test_batched_results_are_complete_when_polled():
    """A ticket is reported only after every field of its result is written
    (status is published last, under the queue lock): polling a batch in
    submission order must never see a terminal status with a partial result."""
    prm = params_rgbd(max_iters=12, stage_iters=(3, 3, 3))
    reqs = _small_requests(200, 12)
    ctx = Context(0, max_slots=16)
    try:
        tks = [ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)[0] for q in reqs]
        outs = [ctx.poll(t) for t in tks]
    finally:
        ctx.close()
    for o in outs:
        assert o["rc"] == 0 and o["iters"] == 12
        assert o["wall_ms"] > 0.0 and o["pairs_within"] > 0 and o["F"] > 0.0
        assert abs(np.linalg.det(o["T"][:3, :3]) - 1.0) < 1e-9


def test_serving_convergence_and_errors():
    ctx = Context(0, hbm_budget=64 << 20, max_slots=4)
    try:
        q = synth.planes_pair(2000, seed=1)
        prm = params_planes(max_iters=200, tol=1e-5)
        tk, _ = ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)
        out = ctx.poll(tk)
        assert out["rc"] == 0 and out["converged"] and 5 < out["iters"] < 200
        ref = ctx.register(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)
        assert ref["iters"] == out["iters"] and np.array_equal(ref["T"], out["T"])
        # the ticket is released once its terminal status has been reported
        assert ctx.poll(tk)["rc"] == CVO_ENOTFOUND
        # a request larger than the device-memory budget fails alone; the
        # scheduler keeps serving the others
        big = synth.rgbd_pair(200000, 200000, seed=6101, select="random")
        tk2, _ = ctx.submit(big.src_xyz, big.src_feat, big.tgt_xyz, big.tgt_feat, prm)
        tk3, _ = ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)
        assert ctx.poll(tk2)["rc"] == CVO_ENOMEM
        again = ctx.poll(tk3)
        assert again["rc"] == 0 and np.array_equal(again["T"], out["T"])
    finally:
        ctx.close()


def test_poll_unknown_ticket_and_pending():
    ctx = Context(0)
    try:
        assert ctx.L.cvo_poll(ctx.h, 12345, 0, None, None) == CVO_ENOTFOUND
        q = synth.rgbd_pair(20000, 20000, seed=6200)
        prm = params_rgbd()
        tk, _ = ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)
        first = ctx.poll(tk, wait_us=0)  # usually still running
        out = first if first is not None else ctx.poll(tk)
        assert out["rc"] == 0 and out["iters"] == 100
        bad = q.src_xyz.copy()
        bad[0, 0] = np.nan
        with pytest.raises(CvoError) as e:
            ctx.submit(bad, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)
        assert e.value.code == CVO_EINVAL
    finally:
        ctx.close()


def test_batched_mixed_kernel_variants_equal_sync():
    """Requests of different kernel variants (precision, label channels,
    cutoff, step rule, value floor) submitted together run in separate
    launch groups and each equals its synchronous run bit for bit."""
    rng = np.random.default_rng(91)
    cases = []
    for k, (prec, fd, kappa, rule, floor) in enumerate([("fp32", 5, 3.0, "fixed", 0.0), ("fp64", 5, 3.0, "fixed", 0.0),
                                                        ("fp32", 3, 3.0, "quartic", 0.0), ("fp32", 5, 0.0, "fixed", 0.0),
                                                        ("fp32", 5, 0.0, "quartic", 1e-3), ("fp64", 2, 3.0, "quartic", 0.0)]):
        q = synth.rgbd_pair(2500 + 300 * k, 2200 + 200 * k, seed=8100 + k)
        sf = q.src_feat[:, :fd].copy()
        tf = q.tgt_feat[:, :fd].copy()
        prm = params_rgbd(max_iters=8, stage_iters=(2, 2, 2), precision=prec, step_rule=rule,
                          cutoff_mult=kappa, kernel_floor=floor)
        cases.append((q, sf, tf, prm))
    ctx = Context(0, max_slots=8)
    try:
        sync = [ctx.register(q.src_xyz, sf, q.tgt_xyz, tf, prm) for q, sf, tf, prm in cases]
        tks = [ctx.submit(q.src_xyz, sf, q.tgt_xyz, tf, prm)[0] for q, sf, tf, prm in cases]
        bat = [ctx.poll(t) for t in tks]
    finally:
        ctx.close()
    for s, b in zip(sync, bat):
        assert b["rc"] == 0 and b["iters"] == 8
        assert np.array_equal(s["T"], b["T"]) and s["F"] == b["F"]
    # the variants differ from one another
    assert len({float(s["F"]) for s in sync}) == len(sync)


def test_serving_counters():
    prm = params_rgbd(max_iters=6, stage_iters=(2, 2, 2))
    reqs = _small_requests(300, 5)
    ctx = Context(0, max_slots=8)
    try:
        s0 = ctx.serving_stats()
        assert s0["completed"] == 0 and s0["active"] == 0 and s0["pending"] == 0
        tks = [ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)[0] for q in reqs]
        bad = ctx.submit(reqs[0].src_xyz, reqs[0].src_feat, reqs[0].tgt_xyz + np.float32(50.0), reqs[0].tgt_feat,
                         prm)[0]
        outs = [ctx.poll(t) for t in tks]
        assert ctx.poll(bad)["rc"] == CVO_ENOOVERLAP
        import time
        t0 = time.time()
        while ctx.serving_stats()["active"] and time.time() - t0 < 10:
            time.sleep(0.01)
        s1 = ctx.serving_stats()
    finally:
        ctx.close()
    assert all(o["rc"] == 0 for o in outs)
    assert s1["completed"] == 6 and s1["failed"] == 1
    assert s1["active"] == 0 and s1["pending"] == 0 and s1["hbm_in_use"] == 0


def test_served_memory_returns_when_idle():
    # a burst that holds several GB at once; once the scheduler has nothing
    # left to run, the memory pool of served requests keeps at most 4 GiB
    import time
    import torch
    dev = torch.device("cuda:0")
    p = synth.rgbd_pair(60000, 60000, seed=5101, select="random")
    t = [torch.from_numpy(a).to(dev) for a in (p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat)]
    torch.cuda.synchronize()
    prm = params_rgbd(max_iters=3, stage_iters=(1, 1, 1))
    ctx = Context(0, max_slots=256)
    try:
        free0 = torch.cuda.mem_get_info()[0]
        tks = [ctx.submit(*t, prm) for _ in range(160)]
        outs = [ctx.poll(tk) for tk, _ in tks]
        peak = ctx.serving_stats()["hbm_peak"]
        t0 = time.time()
        while ctx.serving_stats()["active"] and time.time() - t0 < 20:
            time.sleep(0.01)
        time.sleep(0.5)  # the scheduler trims after its last chunk
        free1 = torch.cuda.mem_get_info()[0]
    finally:
        ctx.close()
    assert all(o["rc"] == 0 for o in outs)
    assert peak > (6 << 30), peak            # the burst did hold more than the pool keeps
    assert free0 - free1 < (4 << 30) + (512 << 20), (free0 - free1, peak)


def test_queue_limit_busy():
    """A bounded submission queue: with no room every submission is refused
    with CVO_EBUSY and nothing is queued; with room again it is accepted."""
    from paper_1904_02266_amd import CVO_EBUSY
    q = synth.planes_pair(500, seed=3)
    prm = params_planes(max_iters=5)
    ctx = Context(0, max_slots=2)
    try:
        ctx.set_queue_limit(0)
        with pytest.raises(CvoError) as e:
            ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)
        assert e.value.code == CVO_EBUSY
        assert ctx.serving_stats()["pending"] == 0
        ctx.set_queue_limit(16)
        tk, _ = ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)
        assert ctx.poll(tk)["rc"] == 0
    finally:
        ctx.close()


def test_batched_ticket_traces():
    """Each batched ticket keeps its own per-iteration trace: readable once
    the request has finished, before and after the poll, and equal to the
    synchronous run's trace."""
    reqs = _small_requests(400, 3)
    prm = params_rgbd(max_iters=9, stage_iters=(3, 3, 3), trace=True)
    ctx = Context(0, max_slots=4)
    try:
        sync = []
        for q in reqs:
            ctx.register(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)
            sync.append(ctx.trace())
        tks = [ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, prm)[0] for q in reqs]
        # the last ticket: wait for it, then read its trace before polling it
        import time
        t0 = time.time()
        tr_last = None
        while tr_last is None and time.time() - t0 < 30:
            tr_last = ctx.trace(ticket=tks[-1])
            time.sleep(0.002)
        outs = [ctx.poll(t) for t in tks]
        after = [ctx.trace(ticket=t) for t in tks]
        with pytest.raises(CvoError) as e:
            ctx.trace(ticket=987654321)
        assert e.value.code == CVO_ENOTFOUND
    finally:
        ctx.close()
    assert all(o["rc"] == 0 for o in outs)
    np.testing.assert_array_equal(tr_last, sync[-1])
    for s, a in zip(sync, after):
        assert a.shape == (9, 26)
        np.testing.assert_array_equal(a, s)


def test_admission_charges_exact_bytes_for_scattered_targets():
    """Targets far apart from one another fall into many small clusters, so
    their iteration buffers outgrow the admission estimate; the scheduler
    charges the exact size once the ingest has counted them, so the
    memory in use never falls below what the requests hold."""
    rng = np.random.default_rng(5)
    m = 4000
    z = (rng.uniform(-1, 1, size=(m, 3)) * 40.0).astype(np.float32)          # sparse: ~5 m apart
    x = (z + rng.normal(0, 0.01, size=z.shape)).astype(np.float32)
    l = rng.uniform(0, 1, size=(m, 5)).astype(np.float32)
    prm = Params(stage_ell=(0.1,), cutoff_mult=3.0, max_iters=20)
    dense = synth.rgbd_pair(4000, 4000, seed=6300)
    ctx = Context(0, max_slots=4)
    try:
        tk1, _ = ctx.submit(x, l, z, l, prm)
        tk2, _ = ctx.submit(dense.src_xyz, dense.src_feat, dense.tgt_xyz, dense.tgt_feat, prm)
        o1, o2 = ctx.poll(tk1), ctx.poll(tk2)
        st = ctx.serving_stats()
    finally:
        ctx.close()
    assert o1["rc"] == 0 and o2["rc"] == 0
    assert o1["device_bytes"] > o2["device_bytes"]      # many clusters
    assert st["hbm_peak"] >= o1["device_bytes"]
    assert st["hbm_in_use"] == 0


def test_exact_size_that_does_not_fit_waits_then_runs():
    """With a budget that holds one scattered request but not two, the
    second waits in the queue (its exact size known) and runs after the
    first; both results equal their synchronous runs."""
    rng = np.random.default_rng(6)
    m = 3000
    reqs = []
    for k in range(2):
        z = (rng.uniform(-1, 1, size=(m, 3)) * 40.0).astype(np.float32)
        x = (z + rng.normal(0, 0.01, size=z.shape)).astype(np.float32)
        l = rng.uniform(0, 1, size=(m, 5)).astype(np.float32)
        reqs.append((x, l, z, l))
    prm = Params(stage_ell=(0.1,), cutoff_mult=3.0, max_iters=10)
    probe = Context(0)
    try:
        sync = [probe.register(*r, prm) for r in reqs]
    finally:
        probe.close()
    one = max(s["device_bytes"] for s in sync)
    ctx = Context(0, hbm_budget=int(one * 1.5), max_slots=4)
    try:
        tks = [ctx.submit(*r, prm)[0] for r in reqs]
        outs = [ctx.poll(t) for t in tks]
        st = ctx.serving_stats()
    finally:
        ctx.close()
    for s, o in zip(sync, outs):
        assert o["rc"] == 0 and np.array_equal(s["T"], o["T"])
    assert st["hbm_peak"] <= int(one * 1.5)


def test_serving_alone_equals_mix_under_poisson_traffic():
    """16 requests of the serving workload (lognormal sizes cut from random
    pixel subsets of 300k frames, conjugate rule, stop at |tau d| < 1e-5,
    cap 200) give bit-identical results when run alone and when submitted at
    Poisson arrival times (rate 1000/s) among other requests."""
    import time
    import torch
    dev = torch.device("cuda:0")
    pool = []
    for k in range(2):
        p = synth.rgbd_pair(300000, 300000, seed=5100 + k, select="random")
        r = np.random.default_rng(5117 + k)
        a, b = r.permutation(len(p.src_xyz)), r.permutation(len(p.tgt_xyz))
        pool.append([torch.from_numpy(np.ascontiguousarray(v)).to(dev)
                     for v in (p.src_xyz[a], p.src_feat[a], p.tgt_xyz[b], p.tgt_feat[b])])
    torch.cuda.synchronize()
    stream = synth.serving_stream(1000, window_s=0.25, seed=55, nmax=60000)
    assert len(stream) > 150
    prm = params_rgbd(max_iters=200, step_rule="conjugate", tol=1e-5)
    chosen = set(range(0, len(stream), max(1, len(stream) // 16))[:16])

    def cut(seed, ns, nt):
        c = pool[seed % 2]
        return c[0][:ns], c[1][:ns], c[2][:nt], c[3][:nt]

    ctx = Context(0, max_slots=256)
    try:
        alone = {}
        for i in sorted(chosen):
            _, seed, ns, nt = stream[i]
            tk, keep = ctx.submit(*cut(seed, ns, nt), prm)
            alone[i] = ctx.poll(tk)
        t0 = time.perf_counter()
        subs = []
        for i, (arr, seed, ns, nt) in enumerate(stream):
            now = time.perf_counter() - t0
            if arr > now:
                time.sleep(arr - now)
            subs.append((i, ctx.submit(*cut(seed, ns, nt), prm)))
        mixed = {i: ctx.poll(tk) for i, (tk, keep) in subs}
        peak_active = ctx.serving_stats()
    finally:
        ctx.close()
    for i in chosen:
        a, m = alone[i], mixed[i]
        assert a["rc"] == 0 and m["rc"] == 0, (i, a["rc"], m["rc"])
        assert a["iters"] == m["iters"] and a["converged"] == m["converged"]
        assert np.array_equal(a["T"], m["T"]) and a["F"] == m["F"], i
    assert sum(m["converged"] for m in mixed.values()) >= 0.9 * len(mixed)
