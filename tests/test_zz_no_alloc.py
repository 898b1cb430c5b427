"""cvo_eval_static (the evaluation that allocates nothing) against cvo_eval.

Both run the same kernels on the same inputs; the static variant takes its
device buffers from the library's per-device array.  Two calls in a row, the
second on smaller clouds (the array keeps the first call's contents), plus
the limit checks.  Results must equal cvo_eval's bit for bit (same kernels,
same reduction order), which is within the C12 tolerance of the oracle that
cvo_eval's own tests establish; the oracle is checked here too.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1904_02266_amd import CVO_ENOMEM, Context, CvoError, Params, synth
from paper_1904_02266_amd._binding import _Cloud, _pose, cvo_cloud

pytestmark = pytest.mark.gpu


def _static_call(ctx, x, lx, z, lz, T, prm):
    """cvo_eval_static through the C ABI (ctypes, no binding helper)."""
    s, t = _Cloud(x, lx), _Cloud(z, lz)
    p, keep = prm.to_c()
    Ta, Tp = _pose(T)
    F = ctypes.c_double()
    w = (ctypes.c_double * 3)()
    v = (ctypes.c_double * 3)()
    rc = ctx.L.cvo_eval_static(ctx.h, ctypes.byref(s.c), ctypes.byref(t.c), ctypes.byref(p), Tp, ctypes.byref(F),
                               w, v)
    return rc, np.array([F.value, *w[:], *v[:]])


def test_static_eval_equals_eval_twice_then_smaller():
    import torch
    ctx = Context(0)
    try:
        big = synth.rgbd_pair(30000, 28000, seed=2)
        small = synth.rgbd_pair(5000, 7000, seed=77)
        dev = torch.device("cuda:0")
        for p, ell in ((big, 0.126), (small, 0.05)):
            T = synth.random_motion(np.random.default_rng(3), 2.0, 0.02) @ p.T_true
            prm = Params(stage_ell=(ell,), cutoff_mult=3.0)
            for on_dev in (False, True):
                arrs = (p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat)
                if on_dev:
                    arrs = tuple(torch.from_numpy(a).to(dev) for a in arrs)
                    torch.cuda.synchronize()
                ref = ctx.eval(*arrs, T, prm)
                rc, got = _static_call(ctx, *arrs, T, prm)
                assert rc == 0, (rc, ctx.L.cvo_last_error(ctx.h))
                np.testing.assert_array_equal(got, ref)
            o = oracle.eval(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, T, ell=ell, kappa=3.0)
            assert abs(got[0] - o["g"][0]) <= 1e-5 * o["g"][0]
            assert (np.abs(got[1:] - o["g"][1:]) <= 1e-5 * o["abs"][1:]).all()
        # brute force (no cutoff) and FP64 through the same array
        q = synth.planes_pair(2000, seed=1)
        for prec in ("fp32", "fp64"):
            prm = Params(stage_ell=(0.1,), precision=prec)
            ref = ctx.eval(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, np.eye(4), prm)
            rc, got = _static_call(ctx, q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, np.eye(4), prm)
            assert rc == 0
            np.testing.assert_array_equal(got, ref)
    finally:
        ctx.close()


def test_static_eval_limits():
    ctx = Context(0)
    try:
        rng = np.random.default_rng(1)
        x = rng.uniform(-1, 1, size=(70000, 3)).astype(np.float32)
        l = rng.uniform(0, 1, size=(70000, 5)).astype(np.float32)
        rc, _ = _static_call(ctx, x, l, x[:100], l[:100], np.eye(4), Params(stage_ell=(0.1,), cutoff_mult=3.0))
        assert rc == CVO_ENOMEM
        assert b"65,536" in ctx.L.cvo_last_error(ctx.h)
        # still usable afterwards
        q = synth.planes_pair(500, seed=2)
        prm = Params(stage_ell=(0.1,))
        rc, got = _static_call(ctx, q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, np.eye(4), prm)
        assert rc == 0
        np.testing.assert_array_equal(got, ctx.eval(q.src_xyz, q.src_feat, q.tgt_xyz, q.tgt_feat, np.eye(4), prm))
    finally:
        ctx.close()
