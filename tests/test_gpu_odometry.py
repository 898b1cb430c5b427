"""Frame-to-frame odometry on a synthetic RGB-D sequence with the TUM
parameter set of Table 1 (front end and registrations on the GPU).

The frames carry 1% depth noise and independent pixel selections, which
bounds the attainable accuracy (about 0.1-0.5 deg and 0.5-3 cm per pair on
1 deg / 2 cm steps); the checks are that the estimates beat the no-motion
estimate and stay within that floor, and that each link of the chain is the
plain registration of its two frames."""
import numpy as np
import pytest

from paper_1904_02266_amd import Context, odometry, params_table1, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frames():
    return synth.rgbd_sequence(7, seed=9)


@pytest.mark.parametrize("init", ["identity", "constant_velocity"])
def test_sequence_relative_errors(frames, init):
    ctx = Context(0)
    try:
        prm = params_table1()
        res = odometry.run_on_device(ctx, frames, prm, init=init)
        # one link again, directly: identical to the chained estimate
        k = 2
        a = ctx.frontend(frames[k].depth, frames[k].rgb, 30000, frames[k].fx, frames[k].fy, frames[k].cx,
                         frames[k].cy, frames[k].dmin, frames[k].dmax)
        b = ctx.frontend(frames[k + 1].depth, frames[k + 1].rgb, 30000, frames[k + 1].fx, frames[k + 1].fy,
                         frames[k + 1].cx, frames[k + 1].cy, frames[k + 1].dmin, frames[k + 1].dmax)
        T0 = np.eye(4) if init == "identity" else res.relative[k - 1]
        direct = ctx.register(a[0], a[1], b[0], b[1], prm, T0=T0)
    finally:
        ctx.close()
    assert np.array_equal(direct["T"], res.relative[k])
    truth = [odometry.pose_errors(np.eye(4), odometry.relative_truth(frames[q].pose, frames[q + 1].pose))
             for q in range(len(frames) - 1)]
    motion_rot = np.array([t[0] for t in truth])
    motion_trans = np.array([t[1] for t in truth])
    assert res.rot_err_deg.mean() < 0.6 * motion_rot.mean(), (res.rot_err_deg, motion_rot)
    assert res.trans_err_m.mean() < 0.9 * motion_trans.mean(), (res.trans_err_m, motion_trans)
    cdf = res.cdf()
    assert cdf["rot_deg"][50] < 0.5 and cdf["trans_m"][50] < 0.02, cdf
    # the chained trajectory is the product of the links
    G = frames[0].pose.copy()
    for T in res.relative:
        G = G @ T
    np.testing.assert_allclose(G, res.trajectory[-1], atol=1e-12)
