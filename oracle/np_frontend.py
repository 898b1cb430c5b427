"""NumPy oracle of the RGB-D front end (TEST INFRASTRUCTURE ONLY).

The step before registration in the paper's RGB-D experiment (Sec. VII-B,
TUM RGB-D benchmark and Table 1): each frame becomes a semi-dense labelled
point cloud by keeping the pixels of high image gradient and taking their
points from the organised depth image (one point per pixel), with the pixel's
colour as its label (the colour remark of Sec. VII-B).

The definition below fixes every floating-point operation that decides which
pixels are kept, in FP32 and in this order, so that a device implementation
can reproduce the selection exactly:

  I      = ((r + g) + b) / 3                         intensity, per pixel
  gu     = (I[v, u+1] - I[v, u-1]) / 2  (interior),  I[v,1] - I[v,0],  I[v,W-1] - I[v,W-2]
  gv     = the same along v (rows)
  s      = gu*gu + gv*gv                             (two products, one sum; no fused multiply-add)
  valid  = depth finite and fl32(dmin) <= depth <= fl32(dmax)
  keep   = the k valid pixels of largest s, ties to the smaller pixel index
           p = v W + u; all valid pixels when there are at most k
  order  = increasing p
  point  = (rx_u d, ry_v d, d), rx_u = fl32((u - cx) / fx), ry_v = fl32((v - cy) / fy)
           (the ray in FP64, rounded once; one FP32 product each)
  label  = (r, g, b, 0.5 + 0.5 tanh(gu / 0.05), 0.5 + 0.5 tanh(gv / 0.05))

(The point's colour and the two gradient channels are the five label
channels of the registration workloads.)  A frame with width or height 1 has
no gradient along that axis (zero).
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def intensity(rgb):
    rgb = np.asarray(rgb, dtype=F32)
    return ((rgb[..., 0] + rgb[..., 1]) + rgb[..., 2]) / F32(3.0)


def gradients(I):
    I = np.asarray(I, dtype=F32)
    H, W = I.shape
    gu = np.zeros_like(I)
    gv = np.zeros_like(I)
    if W >= 2:
        gu[:, 1:-1] = (I[:, 2:] - I[:, :-2]) / F32(2.0)
        gu[:, 0] = I[:, 1] - I[:, 0]
        gu[:, -1] = I[:, -1] - I[:, -2]
    if H >= 2:
        gv[1:-1, :] = (I[2:, :] - I[:-2, :]) / F32(2.0)
        gv[0, :] = I[1, :] - I[0, :]
        gv[-1, :] = I[-1, :] - I[-2, :]
    return gu, gv


def select(depth, s, dmin, dmax, k):
    """Pixel indices kept (increasing), by the definition above."""
    d = np.asarray(depth, dtype=F32).reshape(-1)
    s = np.asarray(s, dtype=F32).reshape(-1)
    with np.errstate(invalid="ignore"):
        valid = np.isfinite(d) & (d >= F32(dmin)) & (d <= F32(dmax))
    idx = np.flatnonzero(valid)
    if idx.size <= k:
        return idx
    order = np.lexsort((idx, -s[idx].astype(np.float64)))   # by s descending, then index
    return np.sort(idx[order[:k]])


def frontend(depth, rgb, fx, fy, cx, cy, dmin, dmax, k):
    """Returns (xyz [n,3] FP32, feat [n,5] FP64, pixel index [n])."""
    depth = np.asarray(depth, dtype=F32)
    H, W = depth.shape
    I = intensity(rgb)
    gu, gv = gradients(I)
    s = gu * gu + gv * gv                      # NumPy: separate products and sum, FP32
    keep = select(depth, s, dmin, dmax, k)
    v, u = np.divmod(keep, W)
    rx = ((u.astype(np.float64) - cx) / fx).astype(F32)
    ry = ((v.astype(np.float64) - cy) / fy).astype(F32)
    d = depth.reshape(-1)[keep]
    xyz = np.stack([rx * d, ry * d, d], axis=1).astype(F32)
    col = np.asarray(rgb, dtype=F32).reshape(-1, 3)[keep].astype(np.float64)
    g1 = gu.reshape(-1)[keep].astype(np.float64)
    g2 = gv.reshape(-1)[keep].astype(np.float64)
    feat = np.concatenate([col, (0.5 + 0.5 * np.tanh(g1 / 0.05))[:, None],
                           (0.5 + 0.5 * np.tanh(g2 / 0.05))[:, None]], axis=1)
    return xyz, feat, keep
