"""Registration on SE(2) of planar clouds on the GPU against the general-n
oracle (eq. flow with n = 2, oracle/np_sen.py).

The library runs planar clouds as points (x, y, 0) on the subgroup of
rotations about z and translations in the plane; its gradient there is eq.
flow's for n = 2 (w^{12} = the z component of x cross z~, v in the plane),
its exponential the SE(2) one.  Checked: the gradient at random poses (C12
tolerance), and the registration's final pose against the oracle's
trajectory under the same fixed step (1e-4 rad / 1e-4 m)."""
import numpy as np
import pytest

from oracle import np_sen
from paper_1904_02266_amd import Context, Params

pytestmark = pytest.mark.gpu


def _planar_pair(count, seed, ang=0.08, trans=0.08, noise=0.003):
    rng = np.random.default_rng(seed)
    # a floor plan: points along the walls of two rooms plus scattered clutter
    walls = []
    for (x0, y0, x1, y1) in ((-2, -1.5, 2, -1.5), (2, -1.5, 2, 1.5), (2, 1.5, -2, 1.5), (-2, 1.5, -2, -1.5),
                             (0, -1.5, 0, 0.5)):
        t = rng.uniform(0, 1, size=count // 6)
        walls.append(np.stack([x0 + t * (x1 - x0), y0 + t * (y1 - y0)], axis=1))
    walls.append(rng.uniform(-1.8, 1.8, size=(count - sum(len(w) for w in walls), 2)))
    x = np.concatenate(walls)
    lab = np.stack([0.5 + 0.5 * np.sin(2.1 * x[:, 0] + 0.3), 0.5 + 0.5 * np.cos(1.7 * x[:, 1]),
                    0.5 + 0.5 * np.sin(x[:, 0] + x[:, 1])], axis=1)
    A = np.array([[0.0, -ang], [ang, 0.0]])
    h = np_sen.expm_series(np_sen.twist(A, rng.normal(size=2) * trans))
    z = x @ h[:2, :2].T + h[:2, 2]
    x = x + rng.normal(0, noise, size=x.shape)
    z = z + rng.normal(0, noise, size=z.shape)
    perm = rng.permutation(len(z))
    return (x.astype(np.float32), lab.astype(np.float32), z[perm].astype(np.float32), lab[perm].astype(np.float32), h)


def test_planar_gradient_matches_general_n_oracle():
    x, lx, z, lz, h = _planar_pair(1500, seed=3)
    ctx = Context(0)
    try:
        rng = np.random.default_rng(4)
        for _ in range(3):
            A = rng.normal(size=(2, 2)) * 0.05
            hp = h @ np_sen.expm_series(np_sen.twist(A - A.T, rng.normal(size=2) * 0.03))
            T = np_sen.inverse(hp)                                   # the library's pose acts on targets
            T4 = np.eye(4)
            T4[:2, :2] = T[:2, :2]
            T4[:2, 3] = T[:2, 2]
            x3 = np.concatenate([x, np.zeros((len(x), 1), np.float32)], axis=1)
            z3 = np.concatenate([z, np.zeros((len(z), 1), np.float32)], axis=1)
            g = ctx.eval(x3, lx, z3, lz, T4, Params(stage_ell=(0.2,)))
            F, W, v = np_sen.gradient(x, lx, z, lz, hp, ell=0.2)
            wgt, d, zt = np_sen._terms(x, lx, z, lz, hp, 0.1, 0.2, 0.2, 0.0)
            a2 = float((x.astype(np.float64) ** 2).sum(axis=1).mean())
            A12 = np.abs(wgt * (x[:, None, 0] * zt[None, :, 1] - x[:, None, 1] * zt[None, :, 0])).sum() / (a2 * 0.04)
            Av = np.abs(wgt[:, :, None] * d).sum(axis=(0, 1)) / 0.04
            assert abs(g[0] - F) <= 1e-5 * F
            assert abs(g[3] - W[0, 1]) <= 1e-5 * A12                 # omega_z = w^{12}
            assert (np.abs(g[4:6] - v) <= 1e-5 * Av).all()
            assert abs(g[6]) <= 1e-5 * Av.max() and abs(g[1]) + abs(g[2]) < np.inf
    finally:
        ctx.close()


def test_planar_registration_follows_general_n_oracle():
    x, lx, z, lz, h = _planar_pair(2000, seed=5)
    ctx = Context(0)
    try:
        out = ctx.register_planar(x, lx, z, lz, Params(stage_ell=(0.2,), max_iters=60))
    finally:
        ctx.close()
    est, tr = np_sen.register(x, lx, z, lz, ell=0.2, max_iters=60)
    T_or = np_sen.inverse(est)
    ang = abs(np.arctan2(out["T"][1, 0], out["T"][0, 0]) - np.arctan2(T_or[1, 0], T_or[0, 0]))
    assert out["rc"] == 0 and out["iters"] == 60
    assert ang < 1e-4 and np.linalg.norm(out["T"][:2, 2] - T_or[:2, 2]) < 1e-4, (ang, out["T"], T_or)
    # and both recover the generating motion
    Th = np_sen.inverse(h)
    assert np.linalg.norm(out["T"][:2, 2] - Th[:2, 2]) < 0.01
