"""Pins of the RGB-D front-end oracle (semi-dense selection and back-projection).

Each test checks the vectorised oracle against something it does not share:
scalar per-pixel loops with the edge rules written out, closed forms (linear
intensity ramps, an isolated bright pixel, fronto-parallel planes), and the
pinhole projection taken the other way.
"""
import numpy as np
import pytest

from oracle import np_frontend as fe
from paper_1904_02266_amd import synth

F32 = np.float32


def _scalar_reference(depth, rgb, fx, fy, cx, cy, dmin, dmax, k):
    """Per-pixel loops over the definition, scalar FP32."""
    H, W = depth.shape
    I = [[F32(0)] * W for _ in range(H)]
    for v in range(H):
        for u in range(W):
            r, g, b = (F32(c) for c in rgb[v, u])
            I[v][u] = F32(F32(F32(r + g) + b) / F32(3))
    rows = []
    for v in range(H):
        for u in range(W):
            if W == 1:
                gu = F32(0)
            elif u == 0:
                gu = F32(I[v][1] - I[v][0])
            elif u == W - 1:
                gu = F32(I[v][W - 1] - I[v][W - 2])
            else:
                gu = F32(F32(I[v][u + 1] - I[v][u - 1]) / F32(2))
            if H == 1:
                gv = F32(0)
            elif v == 0:
                gv = F32(I[1][u] - I[0][u])
            elif v == H - 1:
                gv = F32(I[H - 1][u] - I[H - 2][u])
            else:
                gv = F32(F32(I[v + 1][u] - I[v - 1][u]) / F32(2))
            s = F32(F32(gu * gu) + F32(gv * gv))
            d = F32(depth[v, u])
            ok = bool(np.isfinite(d)) and dmin <= d <= dmax
            rows.append((v * W + u, ok, float(s), gu, gv))
    cand = sorted([r for r in rows if r[1]], key=lambda r: (-r[2], r[0]))
    keep = sorted(r[0] for r in cand[:k])
    return keep


def _tiny_frame(H, W, seed):
    rng = np.random.default_rng(seed)
    depth = rng.uniform(0.3, 6.0, size=(H, W)).astype(F32)
    depth[rng.random((H, W)) < 0.1] = np.nan
    rgb = rng.uniform(0, 1, size=(H, W, 3)).astype(F32)
    # quantised colours make equal gradients (ties) common
    rgb[: H // 2] = np.round(rgb[: H // 2] * 4) / 4
    return depth, rgb


@pytest.mark.parametrize("H,W,k", [(7, 9, 10), (12, 5, 60), (1, 8, 3), (6, 1, 2), (9, 11, 500)])
def test_selection_matches_scalar_loops(H, W, k):
    depth, rgb = _tiny_frame(H, W, H * 100 + W)
    xyz, feat, keep = fe.frontend(depth, rgb, 50.0, 55.0, W / 2, H / 2, 0.5, 5.0, k)
    assert list(keep) == _scalar_reference(depth, rgb, 50.0, 55.0, W / 2, H / 2, 0.5, 5.0, k)
    assert xyz.shape == (len(keep), 3) and feat.shape == (len(keep), 5)


def test_linear_ramp_gradients_and_index_ties():
    # I = 0.3 + a u + b v exactly representable steps: every pixel (edges
    # included) has gu = a, gv = b, so all scores tie and the first k valid
    # pixels in index order are kept
    H, W = 6, 8
    a, b = 1.0 / 64, 1.0 / 128
    u, v = np.meshgrid(np.arange(W), np.arange(H))
    inten = (0.25 + a * u + b * v).astype(F32)
    rgb = np.repeat(inten[..., None], 3, axis=2)
    gu, gv = fe.gradients(fe.intensity(rgb))
    np.testing.assert_array_equal(gu, np.full((H, W), a, F32))
    np.testing.assert_array_equal(gv, np.full((H, W), b, F32))
    depth = np.full((H, W), 2.0, F32)
    depth[0, 1] = np.nan
    depth[1, 0] = 7.0                      # out of range
    _, _, keep = fe.frontend(depth, rgb, 100.0, 100.0, 4.0, 3.0, 0.5, 5.0, 5)
    assert list(keep) == [0, 2, 3, 4, 5]


def test_isolated_bright_pixel():
    # one pixel brighter by h: its four neighbours get |grad| = h/2 (central
    # differences), the pixel itself 0; everything else 0
    H, W, h = 9, 9, 0.75
    rgb = np.full((H, W, 3), 0.125, F32)
    rgb[4, 4] += h
    depth = np.full((H, W), 1.5, F32)
    xyz, feat, keep = fe.frontend(depth, rgb, 100.0, 100.0, 4.0, 4.0, 0.5, 5.0, 4)
    assert list(keep) == [3 * 9 + 4, 4 * 9 + 3, 4 * 9 + 5, 5 * 9 + 4]
    I = fe.intensity(rgb)
    gu, gv = fe.gradients(I)
    assert gu[4, 3] == F32(h / 2) and gu[4, 5] == F32(-h / 2) and gv[3, 4] == F32(h / 2)
    assert gu[4, 4] == 0 and gv[4, 4] == 0
    # labels: colour, then 0.5 + 0.5 tanh(g / 0.05)
    np.testing.assert_allclose(feat[1], [0.125, 0.125, 0.125, 0.5 + 0.5 * np.tanh(h / 2 / 0.05), 0.5])


def test_backprojection_reprojects_to_pixel():
    H, W = 48, 64
    rng = np.random.default_rng(3)
    depth = rng.uniform(0.6, 4.0, size=(H, W)).astype(F32)
    rgb = rng.uniform(0, 1, size=(H, W, 3)).astype(F32)
    fx, fy, cx, cy = 525.0, 520.0, 31.5, 23.5
    xyz, _, keep = fe.frontend(depth, rgb, fx, fy, cx, cy, 0.5, 5.0, 400)
    v, u = np.divmod(keep, W)
    x, y, z = (xyz[:, q].astype(np.float64) for q in range(3))
    np.testing.assert_allclose(fx * x / z + cx, u, atol=1e-4)
    np.testing.assert_allclose(fy * y / z + cy, v, atol=1e-4)
    np.testing.assert_array_equal(xyz[:, 2], depth.reshape(-1)[keep])


def test_fronto_parallel_plane():
    H, W, Z = 10, 12, 2.5
    depth = np.full((H, W), Z, F32)
    rgb = np.random.default_rng(1).uniform(0, 1, size=(H, W, 3)).astype(F32)
    xyz, _, keep = fe.frontend(depth, rgb, 80.0, 80.0, 5.5, 4.5, 0.5, 5.0, H * W)
    assert len(keep) == H * W
    assert np.all(xyz[:, 2] == F32(Z))
    # points on a plane z = Z spaced Z / f apart along x within a row
    row = xyz[keep // W == 3]
    np.testing.assert_allclose(np.diff(row[:, 0]), Z / 80.0, rtol=1e-6)


def test_synthetic_frames_feed_the_pair_workload():
    # the image generator renders the same frames as the cloud generator
    # (same seed, same draw order): the selection of the front end lands on
    # the cloud generator's points up to near-ties of the FP64 score
    src, tgt, G = synth.rgbd_frame_pair(seed=2)
    pair = synth.rgbd_pair(30000, 30000, seed=2)
    np.testing.assert_array_equal(G, pair.T_true)
    xyz, _, keep = fe.frontend(src.depth, src.rgb, src.fx, src.fy, src.cx, src.cy, src.dmin, src.dmax, 30000)
    a = {tuple(p) for p in np.round(xyz.astype(np.float64), 4)}
    b = {tuple(p) for p in np.round(pair.src_xyz.astype(np.float64), 4)}
    assert len(a & b) > 0.99 * 30000
