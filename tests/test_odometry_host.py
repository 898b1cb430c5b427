"""Host logic of the odometry driver (pose chaining and error metrics), with
stand-ins for the front end and the registration."""
from types import SimpleNamespace

import numpy as np

from paper_1904_02266_amd import odometry, synth


def _frames(n, seed=0):
    rng = np.random.default_rng(seed)
    G = np.eye(4)
    out = []
    for _ in range(n):
        out.append(SimpleNamespace(pose=G.copy()))
        G = G @ synth.random_motion(rng, 3.0, 0.05)
    return out


def test_exact_registrations_reproduce_the_trajectory():
    frames = _frames(7)
    res = odometry.run(frames, register=lambda a, b, T0: (odometry.relative_truth(a.pose, b.pose), 3),
                       frontend=lambda f: f)
    for G_est, f in zip(res.trajectory, frames):
        np.testing.assert_allclose(G_est, f.pose, atol=1e-12)
    assert np.all(res.rot_err_deg < 1e-5) and np.all(res.trans_err_m < 1e-12)  # arccos resolution near 0
    assert res.iterations == [3] * 6


def test_errors_measure_a_known_perturbation():
    frames = _frames(5, seed=1)
    P = synth.random_motion(np.random.default_rng(2), 0.0, 0.0)
    ang = 0.7
    P[:3, :3] = synth.rotation_axis_angle([0, 0, 1], np.radians(ang))
    P[:3, 3] = [0.003, 0.0, 0.004]

    def reg(a, b, T0):
        T = odometry.relative_truth(a.pose, b.pose)
        return T @ P, 1

    res = odometry.run(frames, register=reg, frontend=lambda f: f)
    np.testing.assert_allclose(res.rot_err_deg, ang, rtol=1e-9)
    # translation error of T P against T: |R_T t_P|
    np.testing.assert_allclose(res.trans_err_m, 0.005, rtol=1e-9)
    cdf = res.cdf()
    assert abs(cdf["rot_deg"][50] - ang) < 1e-9


def test_constant_velocity_initialisation_passes_the_previous_estimate():
    frames = _frames(4, seed=3)
    seen = []

    def reg(a, b, T0):
        seen.append(T0.copy())
        return odometry.relative_truth(a.pose, b.pose), 1

    odometry.run(frames, register=reg, frontend=lambda f: f, init="constant_velocity")
    np.testing.assert_array_equal(seen[0], np.eye(4))
    np.testing.assert_allclose(seen[2], odometry.relative_truth(frames[1].pose, frames[2].pose))
