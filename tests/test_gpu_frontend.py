"""The RGB-D front end, the value-floor sparsification and the gradient-norm
stop on the GPU, through the C ABI.

Front end: the kept pixels are decided in FP32 exactly as the oracle's
definition, so points must match bit for bit (same pixels, same order, same
products); the two tanh label channels are compared to 1e-6.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import np_frontend as fe
from oracle import np_oracle as npo
from paper_1904_02266_amd import CVO_EINVAL, Context, CvoError, Params, params_rgbd, params_table1, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def _tiny(H, W, seed):
    rng = np.random.default_rng(seed)
    depth = rng.uniform(0.3, 6.0, size=(H, W)).astype(np.float32)
    depth[rng.random((H, W)) < 0.1] = np.nan
    rgb = rng.uniform(0, 1, size=(H, W, 3)).astype(np.float32)
    rgb[: H // 2] = np.round(rgb[: H // 2] * 4) / 4          # ties
    return depth, rgb


def _check(xyz, feat, ref):
    rx, rf, _ = ref
    assert xyz.shape == rx.shape
    assert np.array_equal(xyz, rx)
    if len(rf):
        assert np.abs(feat.astype(np.float64) - rf).max() <= 1e-6


@pytest.mark.parametrize("H,W,k", [(7, 9, 10), (12, 5, 60), (1, 8, 3), (6, 1, 2), (9, 11, 500), (40, 50, 700),
                                   (130, 257, 4000)])
def test_frontend_tiny_frames(ctx, H, W, k):
    depth, rgb = _tiny(H, W, H * 100 + W)
    xyz, feat = ctx.frontend(depth, rgb, k, 50.0, 55.0, W / 2, H / 2, 0.5, 5.0)
    _check(xyz, feat, fe.frontend(depth, rgb, 50.0, 55.0, W / 2, H / 2, 0.5, 5.0, k))


@pytest.mark.parametrize("k", [30000, 300000, 307200])
def test_frontend_vga_frame(ctx, k):
    src, tgt, G = synth.rgbd_frame_pair(seed=2)
    depth = src.depth.copy()
    depth[100:140, 200:260] = np.nan                      # a hole
    depth[300:310, :] = 6.0                               # out of range
    xyz, feat = ctx.frontend(depth, src.rgb, k, src.fx, src.fy, src.cx, src.cy, src.dmin, src.dmax)
    _check(xyz, feat, fe.frontend(depth, src.rgb, src.fx, src.fy, src.cx, src.cy, src.dmin, src.dmax, k))


def test_frontend_device_inputs(ctx):
    import torch
    src, _, _ = synth.rgbd_frame_pair(seed=4)
    dev = torch.device("cuda:0")
    a = ctx.frontend(src.depth, src.rgb, 20000, src.fx, src.fy, src.cx, src.cy)
    b = ctx.frontend(torch.from_numpy(src.depth).to(dev), torch.from_numpy(src.rgb).to(dev), 20000,
                     src.fx, src.fy, src.cx, src.cy)
    torch.cuda.synchronize()
    assert np.array_equal(a[0], b[0].cpu().numpy()) and np.array_equal(a[1], b[1].cpu().numpy())


def test_frontend_errors(ctx):
    depth, rgb = _tiny(8, 8, 3)
    bad = rgb.copy()
    bad[2, 3, 1] = np.inf
    with pytest.raises(CvoError) as e:
        ctx.frontend(depth, bad, 10, 50.0, 50.0, 4.0, 4.0)
    assert e.value.code == CVO_EINVAL
    with pytest.raises(CvoError):
        ctx.frontend(depth, rgb, 10, 0.0, 50.0, 4.0, 4.0)
    with pytest.raises(CvoError):
        ctx.frontend(depth, rgb, 0, 50.0, 50.0, 4.0, 4.0)
    # no valid pixel: an empty cloud
    xyz, feat = ctx.frontend(np.full((8, 8), np.nan, np.float32), rgb, 10, 50.0, 50.0, 4.0, 4.0)
    assert xyz.shape == (0, 3)


def test_frontend_then_register(ctx):
    # image in, pose out: both frames through the device front end, then the
    # registration; the result is the ground-truth motion to the accuracy the
    # noisy frames allow
    src, tgt, G = synth.rgbd_frame_pair(seed=2)
    sx, sf = ctx.frontend(src.depth, src.rgb, 30000, src.fx, src.fy, src.cx, src.cy)
    tx, tf = ctx.frontend(tgt.depth, tgt.rgb, 30000, tgt.fx, tgt.fy, tgt.cx, tgt.cy)
    out = ctx.register(sx, sf, tx, tf, params_rgbd())
    E = out["T"][:3, :3] @ G[:3, :3].T
    assert np.degrees(np.arccos(np.clip((np.trace(E) - 1) / 2, -1, 1))) < 1.0
    assert np.linalg.norm(out["T"][:3, 3] - E @ G[:3, 3]) < 0.04


def test_kernel_floor_equals_distance_cutoff(ctx):
    p = synth.rgbd_pair(5000, 4000, seed=31)
    sigma, floor = 0.1, 1e-3
    kappa = math.sqrt(2.0 * math.log(sigma ** 2 / floor))
    for ell in (0.15, 0.06):
        a = ctx.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, p.T_true,
                     Params(stage_ell=(ell,), kernel_floor=floor))
        b = ctx.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, p.T_true,
                     Params(stage_ell=(ell,), cutoff_mult=kappa))
        assert np.array_equal(a, b)
        ref = oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, p.T_true, ell=ell, kappa=kappa)
        assert abs(a[0] - ref["g"][0]) <= 1e-5 * ref["g"][0]
        for q in range(1, 7):
            assert abs(a[q] - ref["g"][q]) <= 1e-5 * ref["abs"][q]
    # the value floor itself on a small case (NumPy oracle, definition form)
    s = synth.rgbd_pair(900, 800, seed=33)
    g = ctx.eval(s.src_xyz, s.src_feat, s.tgt_xyz, s.tgt_feat, s.T_true, Params(stage_ell=(0.1,), kernel_floor=floor))
    F, w, v = npo.evaluate(s.src_xyz, s.src_feat, s.tgt_xyz, s.tgt_feat, s.T_true, ell=0.1, kernel_floor=floor)
    assert abs(g[0] - F) <= 1e-5 * F
    # omega and v too, each against the sum of its terms' magnitudes (C12)
    wij, d, zt, _ = npo.terms(s.src_xyz, s.src_feat, s.tgt_xyz, s.tgt_feat, s.T_true, ell=0.1, kernel_floor=floor)
    x = s.src_xyz.astype(np.float64)
    a2 = float((x * x).sum(axis=1).mean())
    cross = np.cross(x[:, None, :], zt[None, :, :])                     # x_i x z~_j
    A_w = (np.abs(wij[:, :, None] * cross).sum(axis=(0, 1))) / (a2 * 0.01)
    A_v = (np.abs(wij[:, :, None] * d).sum(axis=(0, 1))) / 0.01
    assert (np.abs(g[1:4] - w) <= 1e-5 * A_w).all(), (g[1:4], w, A_w)
    assert (np.abs(g[4:7] - v) <= 1e-5 * A_v).all(), (g[4:7], v, A_v)
    assert np.count_nonzero(wij) < wij.size          # the floor drops pairs
    with pytest.raises(CvoError):
        ctx.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, p.T_true,
                 Params(stage_ell=(0.1,), kernel_floor=0.02))       # sigma^2 <= floor
    with pytest.raises(CvoError):
        ctx.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, p.T_true,
                 Params(stage_ell=(0.1,), kernel_floor=floor, cutoff_mult=3.0))


def test_gradient_norm_stop(ctx):
    p = synth.rgbd_pair(6000, 6000, seed=37)
    base = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat,
                        params_rgbd(max_iters=40, stage_iters=(5, 5, 5), trace=True))
    tr = ctx.trace()
    gn = np.linalg.norm(tr[:, 1:7], axis=1)
    thr = float(np.min(gn[15:25])) * 1.01            # reached somewhere in the last stage
    out = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat,
                       params_rgbd(max_iters=40, stage_iters=(5, 5, 5), trace=True, grad_tol=thr))
    k = 15 + int(np.argmax(gn[15:] < thr))
    assert out["converged"] and out["iters"] == k + 1
    assert np.array_equal(ctx.trace(), tr[: k + 1])


def test_table1_parameters_register(ctx):
    # the TUM parameter set (quartic step, value floor, Table 1 schedule and
    # both thresholds) on the RGB-D pair
    p = synth.rgbd_pair(30000, 30000, seed=2)
    out = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, params_table1())
    assert out["rc"] == 0 and out["iters"] >= 21
    E = out["T"][:3, :3] @ p.T_true[:3, :3].T
    assert np.degrees(np.arccos(np.clip((np.trace(E) - 1) / 2, -1, 1))) < 1.0
