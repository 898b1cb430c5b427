"""The quartic step rule (Sec. VI-B, eq. fourth) on the GPU against the oracle.

Coefficients F, A1..A4 of the fourth-order model of G(t) = F(h exp(t xi)):
  F:      |F - F_ref| <= 1e-5 F_ref
  A_k:    |A_k - A_ref,k| <= tol * S_k, S_k = sum_ij |term_k,ij| from the oracle
          (A_k cancels between pairs; its error is measured against the size
          of the summed terms), tol = 2e-5 on the FP32 path (the terms of g^3
          and g^4 combine powers of beta computed in FP32), 1e-10 on FP64.
Steps (teacher-forced): at the GPU's pose before iteration k the GPU's
gradient matches the oracle's, and where that gradient is resolved the GPU's
tau equals the oracle's quartic step (see _teacher_forced).  The step kernel
takes A1 = a^2 |omega|^2 + b^2 |v|^2 from the identity along the gradient;
the oracle sums it.
"""
import numpy as np
import pytest

import oracle
from paper_1904_02266_amd import Context, Params, params_planes, params_rgbd, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def rgbd_small():
    return synth.rgbd_pair(6000, 5000, seed=31)


def check_coef(c, ref, absref, tol, what=""):
    ftol = 1e-5 if tol > 1e-8 else tol
    assert abs(c[0] - ref[0]) <= ftol * ref[0], (what, "F", c[0], ref[0])
    for k in range(1, 5):
        assert abs(c[k] - ref[k]) <= tol * absref[k], (what, k, c[k], ref[k], (c[k] - ref[k]) / absref[k])


@pytest.mark.parametrize("ell", [0.2, 0.08, 0.05])
def test_coefficients_rgbd_cutoff(ctx, rgbd_small, ell):
    p = rgbd_small
    rng = np.random.default_rng(int(ell * 1000))
    a2 = oracle.mean_sqnorm(p.src_xyz)
    for trial in range(3):
        T = p.T_true if trial == 0 else synth.random_motion(rng, 3.0, 0.03) @ p.T_true
        g = oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, ell=ell, kappa=3.0, a2=a2)["g"]
        w, v = (g[1:4], g[4:7]) if trial < 2 else (rng.normal(size=3), rng.normal(size=3) * 0.1)
        prm = Params(stage_ell=(ell,), cutoff_mult=3.0)
        c = ctx.quartic(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, w, v, prm)
        ref, absref = oracle.quartic(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, w, v, ell=ell, kappa=3.0)
        check_coef(c, ref, absref, 2e-5, what=f"ell {ell} trial {trial}")


def test_coefficients_planes_brute_force(ctx):
    p = synth.planes_pair(2000, seed=1)
    rng = np.random.default_rng(3)
    for trial in range(3):
        T = np.eye(4) if trial == 0 else synth.random_motion(rng, 8.0, 0.08)
        g = oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, ell=0.1)["g"]
        c = ctx.quartic(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, g[1:4], g[4:7], params_planes())
        ref, absref = oracle.quartic(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, g[1:4], g[4:7], ell=0.1)
        check_coef(c, ref, absref, 2e-5, what=f"trial {trial}")


def test_coefficients_fp64_path(ctx, rgbd_small):
    p = rgbd_small
    T = p.T_true
    g = oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, ell=0.08, kappa=3.0)["g"]
    prm = Params(stage_ell=(0.08,), cutoff_mult=3.0, precision="fp64")
    c = ctx.quartic(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, g[1:4], g[4:7], prm)
    ref, absref = oracle.quartic(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, g[1:4], g[4:7], ell=0.08,
                                 kappa=3.0)
    check_coef(c, ref, absref, 1e-10)


def test_first_coefficient_is_gradient_metric_norm(ctx, rgbd_small):
    # along the GPU's own gradient, A1 = a^2 |omega|^2 + b^2 |v|^2
    p = rgbd_small
    prm = Params(stage_ell=(0.1,), cutoff_mult=3.0, a2=2.0, b2=0.5)
    g = ctx.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, p.T_true, prm)
    c = ctx.quartic(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, p.T_true, g[1:4], g[4:7], prm)
    assert c[0] == g[0]
    A1 = 2.0 * g[1:4] @ g[1:4] + 0.5 * g[4:7] @ g[4:7]
    assert abs(c[1] - A1) <= 1e-4 * A1, (c[1], A1)


def test_zero_direction(ctx, rgbd_small):
    p = rgbd_small
    prm = Params(stage_ell=(0.1,), cutoff_mult=3.0)
    c = ctx.quartic(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, np.eye(4), [0, 0, 0], [0, 0, 0], prm)
    F = ctx.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, np.eye(4), prm)[0]
    assert c[0] == F and np.all(c[1:] == 0.0)


@pytest.mark.parametrize("n,m", [(1, 1), (7, 63), (65, 64), (300, 130), (129, 1)])
def test_coefficients_ragged_sizes(ctx, n, m):
    rng = np.random.default_rng(n * 1000 + m + 7)
    x = rng.uniform(-0.3, 0.3, size=(n, 3)).astype(np.float32)
    z = rng.uniform(-0.3, 0.3, size=(m, 3)).astype(np.float32)
    lx = rng.uniform(0, 1, size=(n, 5)).astype(np.float32)
    lz = rng.uniform(0, 1, size=(m, 5)).astype(np.float32)
    T = synth.random_motion(rng, 5.0, 0.02)
    w, v = rng.normal(size=3), rng.normal(size=3) * 0.2
    for kappa in (0.0, 3.0):
        prm = Params(stage_ell=(0.2,), cutoff_mult=kappa, a2=1.0)
        ref, absref = oracle.quartic(x, lx, z, lz, T, w, v, ell=0.2, kappa=kappa)
        if ref[0] == 0.0:
            continue
        c = ctx.quartic(x, lx, z, lz, T, w, v, prm)
        check_coef(c, ref, absref, 2e-5, what=f"{n}x{m} kappa {kappa}")


def _teacher_forced(ctx, p, prm, kappa, iters, a2):
    """Run the quartic rule on the GPU; at the GPU's pose before each listed
    iteration check the gradient against the oracle, and the step against the
    oracle's quartic step along the oracle's gradient wherever the gradient is
    resolved (its FP32 error bound below 1e-3 of its size: near convergence
    the direction is rounding noise and no step is comparable).  The step's
    tolerance is 1e-4 plus 20 times the direction's relative error bound."""
    out = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, prm)
    tr = ctx.trace()
    assert out["rc"] == 0 and tr.shape[0] == prm.max_iters
    checked = 0
    for k in iters:
        Tk = np.eye(4) if k == 0 else tr[k - 1, 10:26].reshape(4, 4)
        ell = tr[k, 8]
        r = oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, Tk, ell=ell, kappa=kappa, a2=a2)
        g = r["g"]
        assert abs(tr[k, 0] - g[0]) <= 1e-5 * g[0]
        for q in range(1, 7):
            assert abs(tr[k, q] - g[q]) <= 1e-5 * r["abs"][q], (k, q)
        rel = 1e-5 * np.linalg.norm(r["abs"][1:7]) / np.linalg.norm(g[1:7])
        if rel > 1e-3:
            continue
        c, _ = oracle.quartic(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, Tk, g[1:4], g[4:7], ell=ell,
                              kappa=kappa)
        t = oracle.quartic_step(c)
        if t is None:
            t = ell * ell / g[0]
        assert abs(tr[k, 7] - t) <= (1e-4 + 20 * rel) * t, (k, tr[k, 7], t, rel)
        checked += 1
    return out, tr, checked


def test_register_quartic_planes_teacher_forced(ctx):
    p = synth.planes_pair(2000, seed=1)
    prm = params_planes(trace=True, step_rule="quartic", max_iters=30)
    a2 = oracle.mean_sqnorm(p.src_xyz)
    out, tr, checked = _teacher_forced(ctx, p, prm, 0.0, range(30), a2)
    assert checked >= 3
    ref = oracle.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, stage_ell=(0.1,), max_iters=30,
                          step_rule="quartic")
    E = out["T"][:3, :3] @ ref["T"][:3, :3].T
    ang = np.arccos(np.clip((np.trace(E) - 1) / 2, -1, 1))
    assert ang < 1e-4 and np.linalg.norm(out["T"][:3, 3] - E @ ref["T"][:3, 3]) < 1e-4
    # each quartic step raises F
    assert np.all(np.diff(tr[:, 0]) > -1e-6 * tr[1:, 0])


def test_register_quartic_rgbd_schedule_teacher_forced(ctx):
    p = synth.rgbd_pair(4000, 4000, seed=41)
    prm = params_rgbd(max_iters=24, stage_iters=(6, 6, 6), trace=True, step_rule="quartic")
    a2 = oracle.mean_sqnorm(p.src_xyz)
    out, tr, checked = _teacher_forced(ctx, p, prm, 3.0, (0, 1, 6, 7, 12, 13, 18, 19, 23), a2)
    assert checked >= 4
    # the whole trajectory follows the oracle's under the same rule
    ref = oracle.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, kappa=3.0, stage_iters=(6, 6, 6),
                          stage_ell=prm.stage_ell, max_iters=24, step_rule="quartic")
    np.testing.assert_allclose(tr[:, 7], ref["trace"][:, 7], rtol=2e-3)
    E = out["T"][:3, :3] @ ref["T"][:3, :3].T
    assert np.degrees(np.arccos(np.clip((np.trace(E) - 1) / 2, -1, 1))) < 1e-3
    assert np.linalg.norm(out["T"][:3, 3] - E @ ref["T"][:3, 3]) < 1e-4


def test_quartic_rule_batched_equals_sync():
    reqs = [synth.rgbd_pair(3000 + 900 * k, 2800 + 700 * k, seed=7100 + k) for k in range(6)]
    rules = [params_rgbd(max_iters=12, stage_iters=(3, 3, 3), step_rule=r) for r in ("quartic", "fixed", "conjugate")]
    ctx = Context(0, max_slots=8)
    try:
        sync = [ctx.register(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, rules[k % 3]) for k, q in enumerate(reqs)]
        tks = [ctx.submit(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, rules[k % 3])[0] for k, q in enumerate(reqs)]
        bat = [ctx.poll(t) for t in tks]
    finally:
        ctx.close()
    for s, b in zip(sync, bat):
        assert b["rc"] == 0 and b["iters"] == 12
        assert np.array_equal(s["T"], b["T"]) and s["F"] == b["F"]
    assert not np.array_equal(sync[0]["T"], sync[1]["T"])


# --------------------------------------------------------------------------
# conjugate directions (the quartic line search along Polak-Ribiere
# directions): the GPU's trajectory against the oracle's under the same rule
# --------------------------------------------------------------------------
def _angle_deg(A, B):
    E = A[:3, :3] @ B[:3, :3].T
    return float(np.degrees(np.arccos(np.clip((np.trace(E) - 1) / 2, -1, 1))))


def test_register_conjugate_planes_follows_oracle(ctx):
    p = synth.planes_pair(2000, seed=1)
    prm = params_planes(trace=True, step_rule="conjugate", max_iters=30)
    out = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, prm)
    tr = ctx.trace()
    ref = oracle.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, stage_ell=(0.1,), max_iters=30,
                          step_rule="conjugate")
    rt = ref["trace"]
    assert out["rc"] == 0 and tr.shape[0] == 30 and rt.shape[0] == 30
    # the gradient and step of the same iteration: the trajectories agree to
    # FP32 rounding while the gradient is resolved (the first 6 steps: the
    # conjugate directions converge within ~10 and the late directions
    # follow the rounding of a small gradient); then the final pose at the
    # parity bar 1e-4 rad / 1e-4 m (reading C15)
    np.testing.assert_allclose(tr[:10, 0], rt[:10, 0], rtol=1e-5)
    np.testing.assert_allclose(tr[:6, 7], rt[:6, 7], rtol=1e-3)
    assert _angle_deg(out["T"], ref["T"]) < 1e-4 * 180 / np.pi
    assert np.linalg.norm(out["T"][:3, 3] - ref["T"][:3, 3]) < 1e-4
    assert _angle_deg(out["T"], p.T_true) < 0.05


def test_register_conjugate_rgbd_schedule_follows_oracle(ctx):
    p = synth.rgbd_pair(4000, 4000, seed=41)
    prm = params_rgbd(max_iters=24, stage_iters=(6, 6, 6), trace=True, step_rule="conjugate")
    out = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, prm)
    tr = ctx.trace()
    ref = oracle.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, kappa=3.0, stage_iters=(6, 6, 6),
                          stage_ell=prm.stage_ell, max_iters=24, step_rule="conjugate")
    assert out["rc"] == 0 and tr.shape[0] == 24
    np.testing.assert_allclose(tr[:, 0], ref["trace"][:, 0], rtol=1e-5)
    assert _angle_deg(out["T"], ref["T"]) < 1e-4 * 180 / np.pi
    assert np.linalg.norm(out["T"][:3, 3] - ref["T"][:3, 3]) < 1e-4


def test_register_conjugate_converges_with_tolerance(ctx):
    """With tol the conjugate rule stops in the last stage once the applied
    twist is below it.  In that stage the applied twist of both trajectories
    hovers between ~1e-5 and ~2e-4 for some 25 iterations before a step falls
    under the tolerance, so the stopping iteration is a free-running quantity
    (reading C15): the oracle's own moves over 97..101 when the source
    coordinates are jittered by one FP32 ulp, and the GPU's by a few more.
    Asserted: both converge in the last stage within 8 iterations of each
    other, at the same final pose (1e-4 rad / 1e-4 m)."""
    p = synth.rgbd_pair(5000, 5000, seed=43, select="random")
    prm = params_rgbd(max_iters=200, step_rule="conjugate", tol=1e-5)
    out = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, prm)
    ref = oracle.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, kappa=3.0, stage_iters=(25, 25, 25),
                          stage_ell=prm.stage_ell, max_iters=200, step_rule="conjugate", tol=1e-5)
    assert out["rc"] == 0 and out["converged"] and ref["converged"]
    assert 75 < out["iters"] < 200
    assert abs(out["iters"] - ref["iters"]) <= 8, (out["iters"], ref["iters"])
    assert _angle_deg(out["T"], ref["T"]) < 1e-4 * 180 / np.pi
    assert np.linalg.norm(out["T"][:3, 3] - ref["T"][:3, 3]) < 1e-4


@pytest.mark.parametrize("fd", [1, 3, 8])
def test_label_channels_against_oracle(ctx, fd):
    """Every label-channel count the kernels are built for, on an RGB-D pair
    with random labels: the gradient sums with and without the cutoff and the
    quartic sums with it (the folded pair form, whose staged labels carry the
    source's factor), and the FP64 path's gradient and quartic sums at its
    1e-10 bar."""
    p = synth.rgbd_pair(5000, 4500, seed=60 + fd)
    rng = np.random.default_rng(fd)
    lx = rng.uniform(0, 1, (len(p.src_xyz), fd)).astype(np.float32)
    lz = rng.uniform(0, 1, (len(p.tgt_xyz), fd)).astype(np.float32)
    T = synth.random_motion(rng, 3.0, 0.03) @ p.T_true
    a2 = oracle.mean_sqnorm(p.src_xyz)
    for kappa, ell in ((3.0, 0.1), (0.0, 0.1)):
        g = ctx.eval(p.src_xyz, lx, p.tgt_xyz, lz, T, Params(stage_ell=(ell,), cutoff_mult=kappa, a2=a2))
        ref = oracle.eval(p.src_xyz, lx, p.tgt_xyz, lz, T, ell=ell, kappa=kappa, a2=a2)
        assert abs(g[0] - ref["g"][0]) <= 1e-5 * ref["g"][0], (fd, kappa)
        for k in range(1, 7):
            assert abs(g[k] - ref["g"][k]) <= 1e-5 * ref["abs"][k], (fd, kappa, k)
    # every pair term in FP64: the FP64 bar
    g = ctx.eval(p.src_xyz, lx, p.tgt_xyz, lz, T, Params(stage_ell=(0.1,), cutoff_mult=3.0, a2=a2, precision="fp64"))
    ref = oracle.eval(p.src_xyz, lx, p.tgt_xyz, lz, T, ell=0.1, kappa=3.0, a2=a2)
    assert abs(g[0] - ref["g"][0]) <= 1e-10 * ref["g"][0], (fd, "fp64")
    for k in range(1, 7):
        assert abs(g[k] - ref["g"][k]) <= 1e-10 * ref["abs"][k], (fd, "fp64", k)
    w, v = rng.normal(size=3), rng.normal(size=3) * 0.1
    c = ctx.quartic(p.src_xyz, lx, p.tgt_xyz, lz, T, w, v, Params(stage_ell=(0.1,), cutoff_mult=3.0, a2=a2))
    ref, absref = oracle.quartic(p.src_xyz, lx, p.tgt_xyz, lz, T, w, v, ell=0.1, kappa=3.0)
    check_coef(c, ref, absref, 2e-5, what=f"fd {fd}")
    c = ctx.quartic(p.src_xyz, lx, p.tgt_xyz, lz, T, w, v,
                    Params(stage_ell=(0.1,), cutoff_mult=3.0, a2=a2, precision="fp64"))
    check_coef(c, ref, absref, 1e-10, what=f"fd {fd} fp64")


def test_coefficients_cell_list_overflow_compact_cluster(ctx):
    from test_gpu_parity import _compact_overflow_case
    x, lx, z, lz, T, ell = _compact_overflow_case()
    rng = np.random.default_rng(5)
    w, v = rng.normal(size=3), rng.normal(size=3) * 0.05
    c = ctx.quartic(x, lx, z, lz, T, w, v, Params(stage_ell=(ell,), cutoff_mult=3.0, a2=1.0))
    ref, absref = oracle.quartic(x, lx, z, lz, T, w, v, ell=ell, kappa=3.0)
    check_coef(c, ref, absref, 2e-5, what="compact overflow")


def test_coefficients_cell_list_overflow(ctx):
    from test_gpu_parity import _overflow_case
    x, lx, z, lz, T = _overflow_case()
    w, v = np.array([0.5, -1.0, 0.3]), np.array([0.02, 0.01, -0.03])
    c = ctx.quartic(x, lx, z, lz, T, w, v, Params(stage_ell=(0.02,), cutoff_mult=3.0, a2=1.0))
    ref, absref = oracle.quartic(x, lx, z, lz, T, w, v, ell=0.02, kappa=3.0)
    check_coef(c, ref, absref, 2e-5, what="overflow")


def test_register_stage_tolerance_follows_oracle(ctx):
    """Stages that end early on their own convergence (stage_tol): the GPU's
    schedule and stopping iteration follow the oracle's under the same rule."""
    p = synth.rgbd_pair(5000, 5000, seed=43, select="random")
    prm = params_rgbd(max_iters=200, step_rule="conjugate", tol=1e-5, stage_tol=1e-4, trace=True)
    out = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, prm)
    tr = ctx.trace()
    ref = oracle.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, kappa=3.0, stage_iters=(25, 25, 25),
                          stage_ell=prm.stage_ell, max_iters=200, step_rule="conjugate", tol=1e-5, stage_tol=1e-4)
    assert out["rc"] == 0 and out["converged"] and ref["converged"]
    starts = lambda t: [0] + [k for k in range(1, len(t)) if t[k, 8] != t[k - 1, 8]]
    sg, so = starts(tr), starts(ref["trace"])
    assert len(sg) == len(so) == 4
    assert all(abs(a - b) <= 2 for a, b in zip(sg, so)), (sg, so)
    assert out["iters"] < 90 and abs(out["iters"] - ref["iters"]) <= 4, (out["iters"], ref["iters"])
    assert _angle_deg(out["T"], ref["T"]) < 1e-4 * 180 / np.pi
    assert np.linalg.norm(out["T"][:3, 3] - ref["T"][:3, 3]) < 1e-4


def test_quartic_step_stays_in_trusted_interval(ctx):
    """A serving request whose FP32 quartic model near convergence once had a
    spurious maximum far out (tau ~ 1e4, the pose left the overlap): with the
    trusted interval (no target moves farther than ell) it converges and
    follows the oracle under the same rule."""
    p = synth.rgbd_pair(300000, 300000, seed=5102, select="random")
    r = np.random.default_rng(5102 + 17)
    a, b = r.permutation(len(p.src_xyz)), r.permutation(len(p.tgt_xyz))
    sx, sf, tx, tf = p.src_xyz[a][:5581], p.src_feat[a][:5581], p.tgt_xyz[b][:4827], p.tgt_feat[b][:4827]
    prm = params_rgbd(max_iters=200, step_rule="conjugate", tol=1e-5, trace=True)
    out = ctx.register(sx, sf, tx, tf, prm, check=False)
    tr = ctx.trace()
    ref = oracle.register(sx, sf, tx, tf, kappa=3.0, stage_iters=(25, 25, 25), stage_ell=prm.stage_ell,
                          max_iters=200, step_rule="conjugate", tol=1e-5)
    assert out["rc"] == 0 and out["converged"] and ref["converged"], (out["rc"], out["iters"])
    # every step moved the targets by at most ell (the tau column against
    # the interval's bound cannot be read back; the twist's size can)
    assert np.all(tr[:, 7] < 1.0)
    assert abs(out["iters"] - ref["iters"]) <= 4
    assert _angle_deg(out["T"], ref["T"]) < 1e-4 * 180 / np.pi
    assert np.linalg.norm(out["T"][:3, 3] - ref["T"][:3, 3]) < 1e-4
