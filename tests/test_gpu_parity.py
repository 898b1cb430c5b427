"""Parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerance (FP32 pair terms, compensated FP32 partials, FP64 reduction):
  F:          |F - F_ref| <= 1e-5 F_ref               (F is a sum of positive terms)
  omega, v:   |g_k - g_ref,k| <= 1e-5 A_k, A_k = sum_ij |term_k,ij| from the oracle
  (the gradient cancels towards zero near convergence, so its error is measured
  against the magnitude of the summed terms, not against its own value)
  FP64 path:  the same with 1e-10.
Pairs on the cutoff boundary may flip between FP32 and FP64 decisions; pair
counts are compared with a small allowance.
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


def check(g, ref, rtol=1e-5, what=""):
    r = ref["g"]
    A = ref["abs"]
    assert abs(g[0] - r[0]) <= rtol * r[0], (what, "F", g[0], r[0], (g[0] - r[0]) / r[0])
    for k in range(1, 7):
        assert abs(g[k] - r[k]) <= rtol * A[k], (what, k, g[k], r[k], (g[k] - r[k]) / A[k])


def rel_err(g, ref):
    r, A = ref["g"], ref["abs"]
    return max([abs(g[0] - r[0]) / r[0]] + [abs(g[k] - r[k]) / A[k] for k in range(1, 7)])


@pytest.fixture(scope="module")
def planes():
    return synth.planes_pair(2000, seed=1)


@pytest.fixture(scope="module")
def rgbd_small():
    return synth.rgbd_pair(6000, 5000, seed=31)


def test_two_point_golden(ctx):
    """The hand-derived two-point case (tests/golden/two_point.json, eq.
    scalar and eq. 3_gradient with the kernel of Sec. IV) through the C ABI:
    F = 1e-3, omega = (0, 0, 0.016 ln 2), v = (0, 0.016 ln 2, 0), with and
    without the cutoff, in both precisions.  The zero components are exact:
    in the target's frame the pair's offset has no x or z part."""
    import json
    import math
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "two_point.json")))
    x = np.array(g["src_xyz"], np.float32)
    lx = np.array(g["src_feat"], np.float32)
    z = np.array(g["tgt_xyz"], np.float32)
    lz = np.array(g["tgt_feat"], np.float32)
    ell = math.sqrt(g["ell_sq_times_2ln2"] / (2.0 * math.log(2.0)))
    c = 0.016 * math.log(2.0)
    for kappa in (3.0, 0.0):
        for precision, rtol in (("fp32", 1e-6), ("fp64", 1e-12)):
            r = ctx.eval(x, lx, z, lz, np.eye(4), Params(stage_ell=(ell,), cutoff_mult=kappa, a2=g["a2"], b2=g["b2"],
                                                          sigma=g["sigma"], feat_scale=g["feat_scale"],
                                                          precision=precision))
            what = (kappa, precision)
            assert abs(r[0] - g["F"]) <= rtol * g["F"], (what, r[0])
            assert abs(r[3] - c) <= rtol * c and abs(r[5] - c) <= rtol * c, (what, r[3], r[5])
            assert r[1] == 0.0 and r[2] == 0.0 and r[4] == 0.0 and r[6] == 0.0, (what, r)


def test_eval_planes_brute_force(ctx, planes):
    p = planes
    rng = np.random.default_rng(0)
    for trial in range(4):
        T = np.eye(4) if trial == 0 else synth.random_motion(rng, 10.0, 0.1)
        g = ctx.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, params_planes())
        ref = oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, ell=0.1)
        check(g, ref, what=f"trial {trial}")


@pytest.mark.parametrize("ell", [0.2, 0.08, 0.05])
def test_eval_rgbd_cutoff(ctx, rgbd_small, ell):
    p = rgbd_small
    T = synth.random_motion(np.random.default_rng(3), 3.0, 0.03) @ p.T_true
    prm = Params(stage_ell=(ell,), cutoff_mult=3.0)
    g = ctx.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, prm)
    ref = oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, ell=ell, kappa=3.0)
    check(g, ref, what=f"ell {ell}")


def test_eval_fp64_path(ctx, rgbd_small):
    p = rgbd_small
    T = p.T_true
    for kappa, ell in ((3.0, 0.1), (0.0, 0.15)):
        prm = Params(stage_ell=(ell,), cutoff_mult=kappa, precision="fp64")
        g = ctx.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, prm)
        ref = oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, ell=ell, kappa=kappa)
        check(g, ref, rtol=1e-10, what=f"fp64 kappa {kappa}")


def test_eval_targets_match_oracle(ctx, rgbd_small):
    p = rgbd_small
    T = p.T_true
    prm = Params(stage_ell=(0.1,), cutoff_mult=3.0)
    sel = np.random.default_rng(5).choice(p.tgt_xyz.shape[0], 64, replace=False).astype(np.int32)
    out = ctx.eval_targets(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, prm, sel=sel)
    ref = oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, ell=0.1, kappa=3.0, sel=sel,
                      per_target=True)
    pt = ref["per_target"]
    for k in range(64):
        if pt[k, 0] == 0.0:
            assert out[k, 0] == 0.0
            continue
        assert abs(out[k, 0] - pt[k, 0]) <= 2e-5 * pt[k, 0], (k, out[k], pt[k])
    # the sum over all targets is the objective
    allt = ctx.eval_targets(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, prm)
    g = ctx.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, prm)
    # different work splits round differently in FP32; both are within the parity bound
    np.testing.assert_allclose(allt.sum(axis=0)[0], g[0], rtol=1e-6)


def test_pair_counts(ctx, rgbd_small):
    p = rgbd_small
    T = p.T_true
    prm = params_rgbd(max_iters=1, stage_ell=(0.1,), stage_iters=())
    out = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, prm, T0=T)
    ref = oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, ell=0.1, kappa=3.0)
    assert abs(out["pairs_within"] - ref["within"]) <= 20, (out["pairs_within"], ref["within"])
    assert out["pairs_examined"] >= out["pairs_within"]


def test_register_planes_trajectory(ctx, planes):
    """Config-1 registration (2,000 points, brute force, 50 steps): teacher-forced
    per-iteration parity and final-pose parity against the oracle trajectory."""
    p = planes
    prm = params_planes(trace=True)
    out = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, prm)
    tr = ctx.trace()
    assert out["iters"] == 50 and tr.shape == (50, 26)
    ref = oracle.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, stage_ell=(0.1,), max_iters=50)
    E = out["T"][:3, :3] @ ref["T"][:3, :3].T
    ang = np.arccos(np.clip((np.trace(E) - 1) / 2, -1, 1))
    assert ang < 1e-4 and np.linalg.norm(out["T"][:3, 3] - E @ ref["T"][:3, 3]) < 1e-4
    # teacher forcing: the oracle at the GPU's pose before each step
    a2 = oracle.mean_sqnorm(p.src_xyz)
    Tk = np.eye(4)
    for k in (0, 1, 10, 49):
        if k > 0:
            Tk = tr[k - 1, 10:26].reshape(4, 4)
        r = oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, Tk, ell=0.1, a2=a2)
        check(tr[k, :7], r, what=f"iter {k}")


def test_register_rgbd_schedule_small(ctx):
    p = synth.rgbd_pair(4000, 4000, seed=41)
    prm = params_rgbd(max_iters=40, stage_iters=(10, 10, 10), trace=True)
    out = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, prm)
    tr = ctx.trace()
    ref = oracle.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, kappa=3.0,
                          stage_iters=(10, 10, 10), stage_ell=prm.stage_ell, max_iters=40)
    np.testing.assert_allclose(tr[:, 8], ref["trace"][:, 8])  # same stage schedule
    E = out["T"][:3, :3] @ ref["T"][:3, :3].T
    ang = np.arccos(np.clip((np.trace(E) - 1) / 2, -1, 1))
    assert ang < 1e-4, ang
    assert np.linalg.norm(out["T"][:3, 3] - E @ ref["T"][:3, 3]) < 1e-4


def test_deterministic_reruns(ctx, rgbd_small):
    p = rgbd_small
    prm = params_rgbd(max_iters=12, stage_iters=(3, 3, 3))
    a = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, prm)
    b = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, prm)
    assert np.array_equal(a["T"], b["T"]) and a["F"] == b["F"]


@pytest.mark.parametrize("n,m", [(1, 1), (7, 63), (65, 64), (300, 130), (129, 1)])
def test_ragged_sizes(ctx, n, m):
    rng = np.random.default_rng(n * 1000 + m)
    x = rng.uniform(-0.3, 0.3, size=(n, 3)).astype(np.float32)
    z = rng.uniform(-0.3, 0.3, size=(m, 3)).astype(np.float32)
    lx = rng.uniform(0, 1, size=(n, 5)).astype(np.float32)
    lz = rng.uniform(0, 1, size=(m, 5)).astype(np.float32)
    T = synth.random_motion(rng, 5.0, 0.02)
    for kappa in (0.0, 3.0):
        prm = Params(stage_ell=(0.2,), cutoff_mult=kappa, a2=1.0)
        g = ctx.eval(x, lx, z, lz, T, prm)
        ref = oracle.eval(x, lx, z, lz, T, ell=0.2, kappa=kappa, a2=1.0)
        if ref["g"][0] == 0.0:
            assert g[0] == 0.0
        else:
            check(g, ref, what=f"{n}x{m} kappa {kappa}")


@pytest.mark.parametrize("n,m", [(1024, 1024), (1025, 2047), (2048, 1023), (3071, 2049)])
def test_sizes_at_sort_tile_boundaries(ctx, n, m):
    # the set-up sorts keys in tiles of 1,024 elements: sizes at and just past
    # tile boundaries, with a cutoff (several cells) and without
    rng = np.random.default_rng(n * 7 + m)
    x = rng.uniform(-0.6, 0.6, size=(n, 3)).astype(np.float32)
    z = (x[rng.integers(0, n, size=m)] + rng.normal(0, 0.02, size=(m, 3))).astype(np.float32)
    lx = rng.uniform(0, 1, size=(n, 5)).astype(np.float32)
    lz = rng.uniform(0, 1, size=(m, 5)).astype(np.float32)
    T = synth.random_motion(rng, 4.0, 0.02)
    for kappa in (0.0, 3.0):
        prm = Params(stage_ell=(0.05,), cutoff_mult=kappa, a2=1.0)
        g = ctx.eval(x, lx, z, lz, T, prm)
        ref = oracle.eval(x, lx, z, lz, T, ell=0.05, kappa=kappa, a2=1.0)
        check(g, ref, what=f"{n}x{m} kappa {kappa}")


def test_duplicate_points_and_single_cell(ctx):
    # every source at one of two points (two keys with hundreds of duplicates
    # each), then every source at the same point (a single cell)
    rng = np.random.default_rng(91)
    n, m = 1500, 700
    base = np.array([[0.1, -0.2, 0.3], [0.14, -0.2, 0.31]], np.float32)
    lx = rng.uniform(0, 1, size=(n, 5)).astype(np.float32)
    lz = rng.uniform(0, 1, size=(m, 5)).astype(np.float32)
    z = (base[0] + rng.normal(0, 0.05, size=(m, 3))).astype(np.float32)
    for pts in (base[rng.integers(0, 2, size=n)], np.repeat(base[:1], n, axis=0)):
        x = np.ascontiguousarray(pts, dtype=np.float32)
        for kappa in (0.0, 3.0):
            prm = Params(stage_ell=(0.03,), cutoff_mult=kappa, a2=1.0)
            g = ctx.eval(x, lx, z, lz, np.eye(4), prm)
            ref = oracle.eval(x, lx, z, lz, np.eye(4), ell=0.03, kappa=kappa, a2=1.0)
            check(g, ref, what=f"duplicates kappa {kappa}")


@pytest.mark.parametrize("fd", [1, 3, 8])
def test_feature_dims(ctx, fd):
    rng = np.random.default_rng(fd)
    x = rng.uniform(-1, 1, size=(700, 3)).astype(np.float32)
    z = (x + rng.normal(0, 0.02, size=x.shape)).astype(np.float32)
    lx = rng.uniform(0, 1, size=(700, fd)).astype(np.float32)
    lz = rng.uniform(0, 1, size=(700, fd)).astype(np.float32)
    for kappa in (0.0, 3.0):
        prm = Params(stage_ell=(0.1,), cutoff_mult=kappa)
        g = ctx.eval(x, lx, z, lz, np.eye(4), prm)
        ref = oracle.eval(x, lx, z, lz, np.eye(4), ell=0.1, kappa=kappa)
        check(g, ref, what=f"fd {fd}")


def test_errors(ctx, rgbd_small):
    from paper_1904_02266_amd import CVO_EINVAL, CVO_ENOOVERLAP, CvoError
    p = rgbd_small
    bad = p.src_xyz.copy()
    bad[5, 2] = np.inf
    with pytest.raises(CvoError) as e:
        ctx.eval(bad, p.src_feat, p.tgt_xyz, p.tgt_feat, np.eye(4), Params())
    assert e.value.code == CVO_EINVAL
    with pytest.raises(CvoError) as e:
        ctx.eval(p.src_xyz, p.src_feat[:, :3], p.tgt_xyz, p.tgt_feat, np.eye(4), Params())
    assert e.value.code == CVO_EINVAL
    with pytest.raises(CvoError) as e:
        ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, Params(stage_ell=(-1.0,)))
    assert e.value.code == CVO_EINVAL
    far = p.tgt_xyz + np.float32(50.0)
    out = ctx.register(p.src_xyz, p.src_feat, far, p.tgt_feat, params_rgbd(max_iters=3, stage_iters=(1, 1, 1)),
                       check=False)
    assert out["rc"] == CVO_ENOOVERLAP and out["iters"] == 0


def test_size_and_schedule_limits(ctx):
    # the largest accepted sizes are checked before any input is read: a
    # point count above 16,000,000, feature dimensions outside 1..8 and more
    # than 8 length-scale stages are rejected (small buffers stand behind the
    # counts; nothing is dereferenced for a rejected request)
    import ctypes
    from paper_1904_02266_amd import CVO_EINVAL, _binding
    L = _binding.load()
    xyz = np.random.default_rng(5).uniform(-0.1, 0.1, size=(4, 3)).astype(np.float32)
    feat = np.full((4, 8), 0.5, np.float32)

    def cloud(n, fd):
        return _binding.cvo_cloud(n, fd, xyz.ctypes.data, feat.ctypes.data, 0)

    T = (ctypes.c_double * 16)(*np.eye(4).ravel())
    F = ctypes.c_double()
    w = (ctypes.c_double * 3)()
    v = (ctypes.c_double * 3)()

    def rc(src, tgt, prm):
        p, keep = prm.to_c()
        return L.cvo_eval(ctx.h, ctypes.byref(src), ctypes.byref(tgt), ctypes.byref(p), T, ctypes.byref(F), w, v)

    ok = Params(stage_ell=(0.1,), a2=1.0)
    assert rc(cloud(4, 5), cloud(4, 5), ok) == 0
    assert rc(cloud(16_000_001, 5), cloud(4, 5), ok) == CVO_EINVAL
    assert rc(cloud(4, 5), cloud(16_000_001, 5), ok) == CVO_EINVAL
    assert rc(cloud(0, 5), cloud(4, 5), ok) == CVO_EINVAL
    assert rc(cloud(4, 9), cloud(4, 9), ok) == CVO_EINVAL
    assert rc(cloud(4, 0), cloud(4, 0), ok) == CVO_EINVAL
    assert rc(cloud(4, 8), cloud(4, 8), ok) == 0
    nine = Params(stage_ell=tuple(0.1 for _ in range(9)), stage_iters=tuple(1 for _ in range(8)), a2=1.0)
    assert rc(cloud(4, 5), cloud(4, 5), nine) == CVO_EINVAL
    eight = Params(stage_ell=tuple(0.1 for _ in range(8)), stage_iters=tuple(1 for _ in range(7)), a2=1.0)
    assert rc(cloud(4, 5), cloud(4, 5), eight) == 0


def test_device_inputs_same_as_host(ctx, rgbd_small):
    import torch
    p = rgbd_small
    dev = torch.device("cuda:0")
    prm = params_rgbd(max_iters=8, stage_iters=(2, 2, 2))
    a = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, prm)
    b = ctx.register(torch.from_numpy(p.src_xyz).to(dev), torch.from_numpy(p.src_feat).to(dev),
                     torch.from_numpy(p.tgt_xyz).to(dev), torch.from_numpy(p.tgt_feat).to(dev), prm)
    assert np.array_equal(a["T"], b["T"])


def _overflow_case():
    # 64 targets on a 3 m line (one cluster) over a dense slab of sources:
    # the cluster's reachable cells (~2,600 at ell = 0.02) exceed the 512-entry
    # cell list, so the pair kernel enumerates the candidate box itself
    rng = np.random.default_rng(77)
    n = 20000
    x = np.stack([rng.uniform(0, 3.0, n), rng.uniform(-0.06, 0.06, n), rng.uniform(-0.06, 0.06, n)], 1)
    z = np.stack([np.linspace(0.0, 3.0, 64), np.zeros(64), np.zeros(64)], 1)
    lx = rng.uniform(0, 1, (n, 5))
    lz = rng.uniform(0, 1, (64, 5))
    T = synth.random_motion(rng, 0.5, 0.005)
    return (x.astype(np.float32), lx.astype(np.float32), z.astype(np.float32), lz.astype(np.float32), T)


def _compact_overflow_case():
    # 64 targets in a cube of half-width 2.95 ell at ell = 0.02 (2.5 of the
    # frame's scaled units, so the cluster takes the expanded, folded pair
    # form), eight of them at its corners, over a dense cube of sources:
    # about 665 reachable non-empty cells, beyond the 512-entry cell list
    rng = np.random.default_rng(78)
    ell = 0.02
    x = rng.uniform(-0.4, 0.4, (60000, 3))
    z = rng.uniform(-2.95 * ell, 2.95 * ell, (64, 3))
    z[:8] = np.array([[a, b, c] for a in (-1, 1) for b in (-1, 1) for c in (-1, 1)]) * 2.95 * ell
    lx = rng.uniform(0, 1, (len(x), 5))
    lz = rng.uniform(0, 1, (64, 5))
    T = synth.random_motion(rng, 0.5, 0.005)
    return (x.astype(np.float32), lx.astype(np.float32), z.astype(np.float32), lz.astype(np.float32), T, ell)


def test_cell_list_overflow_compact_cluster(ctx):
    x, lx, z, lz, T, ell = _compact_overflow_case()
    prm = Params(stage_ell=(ell,), cutoff_mult=3.0, a2=1.0)
    g = ctx.eval(x, lx, z, lz, T, prm)
    ref = oracle.eval(x, lx, z, lz, T, ell=ell, kappa=3.0, a2=1.0)
    check(g, ref, what="compact overflow")
    per = ctx.eval_targets(x, lx, z, lz, T, prm)
    check(per.sum(axis=0), ref, what="compact overflow targets")


def test_cell_list_overflow_path(ctx):
    x, lx, z, lz, T = _overflow_case()
    for ell in (0.02, 0.04):
        g = ctx.eval(x, lx, z, lz, T, Params(stage_ell=(ell,), cutoff_mult=3.0, a2=1.0))
        ref = oracle.eval(x, lx, z, lz, T, ell=ell, kappa=3.0, a2=1.0)
        check(g, ref, what=f"overflow ell {ell}")
        # the per-target path (one work item per cluster) sums in another
        # order: the same bar against the oracle
        per = ctx.eval_targets(x, lx, z, lz, T, Params(stage_ell=(ell,), cutoff_mult=3.0, a2=1.0))
        check(per.sum(axis=0), ref, what=f"overflow targets ell {ell}")


def test_far_from_origin(ctx):
    # clouds 2 km from the origin: the FP64 frames keep the FP32 pair terms
    # as accurate as near the origin (absolute FP32 coordinates there would
    # carry ~1e-4 m of rounding)
    p = synth.rgbd_pair(4000, 3500, seed=43)
    off = np.array([1500.0, -800.0, 1200.0], dtype=np.float32)
    sx = (p.src_xyz + off).astype(np.float32)
    tx = (p.tgt_xyz + off).astype(np.float32)
    T = p.T_true.copy()
    T[:3, 3] += off.astype(np.float64) - T[:3, :3] @ off.astype(np.float64)  # the same motion about the offset
    for kappa in (3.0, 0.0):
        prm = Params(stage_ell=(0.1,), cutoff_mult=kappa, a2=4.0)
        g = ctx.eval(sx, p.src_feat, tx, p.tgt_feat, T, prm)
        ref = oracle.eval(sx, p.src_feat, tx, p.tgt_feat, T, ell=0.1, kappa=kappa, a2=4.0)
        check(g, ref, what=f"far kappa {kappa}")


@pytest.mark.parametrize("mask", [0x1C, 0x07, 0x38])
def test_subgroup_registration_matches_oracle(ctx, mask):
    """Registration on a subgroup of SE(3) (planar motion, rotations,
    translations): the GPU trajectory follows the oracle's and stays in the
    subgroup."""
    p = synth.planes_pair(1500, seed=5)
    prm = Params(stage_ell=(0.1,), max_iters=30, trace=True, dof_mask=mask)
    out = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, prm)
    tr = ctx.trace()
    ref = oracle.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, stage_ell=(0.1,), max_iters=30,
                          dof_mask=mask)
    E = out["T"][:3, :3] @ ref["T"][:3, :3].T
    assert np.arccos(np.clip((np.trace(E) - 1) / 2, -1, 1)) < 1e-4
    assert np.linalg.norm(out["T"][:3, 3] - E @ ref["T"][:3, 3]) < 1e-4
    T = out["T"]
    if mask == 0x1C:
        assert np.all(np.abs(T[2, :2]) < 1e-12) and np.all(np.abs(T[:2, 2]) < 1e-12) and abs(T[2, 3]) < 1e-12
    if mask == 0x07:
        assert np.all(np.abs(T[:3, 3]) < 1e-12)
    if mask == 0x38:
        assert np.all(np.abs(T[:3, :3] - np.eye(3)) < 1e-12)
    a2 = oracle.mean_sqnorm(p.src_xyz)
    for k in (0, 5, 29):
        Tk = np.eye(4) if k == 0 else tr[k - 1, 10:26].reshape(4, 4)
        check(tr[k, :7], oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, Tk, ell=0.1, a2=a2),
              what=f"mask {mask:#x} iter {k}")
