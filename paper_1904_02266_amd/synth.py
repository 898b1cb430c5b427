"""Seeded synthetic inputs for continuous sensor registration.

This module only draws inputs: point clouds with colour-like labels, rigid
motions and request streams.  It holds none of the registration arithmetic
(no kernel, no gradient, no exponential map) so that the CPU oracle and the
GPU library can both consume it without sharing any of the method.

Scenes stand in for the paper's RGB-D workload (Section VII-B: Kinect-class
VGA frames, indoor piecewise-planar scenes, semi-dense high-gradient point
selection, colour labels in R^3).  The dataset itself is not used.

Label model (5 channels, all in [0, 1]):
  * three colour channels c_k(p) = 0.5 + 0.5 sin(2 pi f_k . p + phi_k),
    evaluated at the world surface point p, f_k ~ N(0, (0.4 m^-1)^2 I_3),
    phi_k ~ U[0, 2 pi);
  * two gradient channels of the intensity I = mean_k c_k.
Labels travel with the surface point, so both frames carry the same label for
the same world point (no label noise).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FEAT_DIM = 5

# Pinhole camera for a Kinect-class VGA sensor (project choice).
CAM_W, CAM_H = 640, 480
CAM_F = 525.0
CAM_CX, CAM_CY = 319.5, 239.5


# --------------------------------------------------------------------------
# rigid motions
# --------------------------------------------------------------------------
def _skew(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def rotation_axis_angle(axis, angle):
    """Rodrigues rotation matrix (input generation only)."""
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    K = _skew(axis)
    return np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)


def _unit_vector(rng):
    v = rng.standard_normal(3)
    n = np.linalg.norm(v)
    while n < 1e-12:
        v = rng.standard_normal(3)
        n = np.linalg.norm(v)
    return v / n


def random_motion(rng, theta_max_deg, t_max):
    """4x4 FP64 rigid motion: axis uniform on S^2, angle U[0, theta_max],
    translation direction uniform, magnitude U[0, t_max]."""
    axis = _unit_vector(rng)
    angle = rng.uniform(0.0, math.radians(theta_max_deg))
    tdir = _unit_vector(rng)
    tmag = rng.uniform(0.0, t_max)
    M = np.eye(4)
    M[:3, :3] = rotation_axis_angle(axis, angle)
    M[:3, 3] = tdir * tmag
    return M


def invert_rigid(M):
    Mi = np.eye(4)
    R = M[:3, :3]
    Mi[:3, :3] = R.T
    Mi[:3, 3] = -R.T @ M[:3, 3]
    return Mi


# --------------------------------------------------------------------------
# labels
# --------------------------------------------------------------------------
@dataclass
class Texture:
    freq: np.ndarray   # [3 channels, 3 axes], m^-1
    phase: np.ndarray  # [3]

    @staticmethod
    def draw(rng):
        return Texture(freq=rng.normal(0.0, 0.4, size=(3, 3)),
                       phase=rng.uniform(0.0, 2.0 * math.pi, size=3))

    def colour(self, p):
        """[N,3] colour channels at world points p [N,3]."""
        arg = 2.0 * math.pi * (p @ self.freq.T) + self.phase
        return 0.5 + 0.5 * np.sin(arg)

    def intensity_grad(self, p):
        """Spatial gradient of I = mean_k c_k at p, [N,3] in m^-1."""
        arg = 2.0 * math.pi * (p @ self.freq.T) + self.phase      # [N,3]
        dc = 0.5 * np.cos(arg)[:, :, None] * (2.0 * math.pi * self.freq)[None, :, :]
        return dc.mean(axis=1)


# --------------------------------------------------------------------------
# config 1: three orthogonal planes (room corner), brute force
# --------------------------------------------------------------------------
@dataclass
class CloudPair:
    src_xyz: np.ndarray      # [N,3] float32
    src_feat: np.ndarray     # [N,F] float32
    tgt_xyz: np.ndarray      # [M,3] float32
    tgt_feat: np.ndarray     # [M,F] float32
    T_true: np.ndarray       # [4,4] float64, maps target points onto source points
    meta: dict = field(default_factory=dict)


def planes_pair(n=2000, seed=1, noise=0.005, theta_max_deg=10.0, t_max=0.1,
                half=2.0):
    """Room corner in [-half, half]^3: the faces x=-half, y=-half, z=-half.

    Source: n points uniform over the three faces (split as evenly as
    possible) plus N(0, noise) per coordinate.  Target: the same surface
    points moved by a seeded rigid motion M, fresh noise, seeded permutation.
    The registration answer is T_true = M^-1.
    """
    rng = np.random.default_rng(seed)
    tex = Texture.draw(rng)
    counts = [n // 3 + (1 if k < n % 3 else 0) for k in range(3)]
    pts, gu, gv = [], [], []
    for face, cnt in enumerate(counts):
        uv = rng.uniform(-half, half, size=(cnt, 2))
        p = np.empty((cnt, 3))
        axes = [a for a in range(3) if a != face]   # in-plane axes in axis order
        p[:, face] = -half
        p[:, axes[0]] = uv[:, 0]
        p[:, axes[1]] = uv[:, 1]
        g = tex.intensity_grad(p)
        pts.append(p)
        gu.append(g[:, axes[0]])
        gv.append(g[:, axes[1]])
    surf = np.concatenate(pts)
    gu = np.concatenate(gu)
    gv = np.concatenate(gv)
    feat = np.concatenate([tex.colour(surf),
                           (0.5 + 0.5 * np.tanh(gu / 2.0))[:, None],
                           (0.5 + 0.5 * np.tanh(gv / 2.0))[:, None]], axis=1)
    src = surf + rng.normal(0.0, noise, size=surf.shape)
    M = random_motion(rng, theta_max_deg, t_max)
    moved = surf @ M[:3, :3].T + M[:3, 3]
    tgt = moved + rng.normal(0.0, noise, size=surf.shape)
    perm = rng.permutation(n)
    return CloudPair(src.astype(np.float32), feat.astype(np.float32),
                     tgt[perm].astype(np.float32), feat[perm].astype(np.float32),
                     invert_rigid(M),
                     dict(kind="planes", seed=seed, n=n, M=M))


# --------------------------------------------------------------------------
# configs 2-5: synthetic RGB-D frames of a piecewise-planar room
# --------------------------------------------------------------------------
@dataclass
class Room:
    lo: np.ndarray            # room box (interior) min corner, world frame
    hi: np.ndarray
    boxes: list               # list of (lo, hi) solid axis-aligned boxes
    tex: Texture

    @staticmethod
    def draw(rng):
        # 6 m wide (x), 3 m high (y, pointing down), 6 m deep (z); the source
        # camera sits at the origin looking along +z, 1.5 m above the floor.
        lo = np.array([-3.0, -1.5, -1.5])
        hi = np.array([3.0, 1.5, 4.5])
        boxes = []
        for _ in range(3):
            size = rng.uniform(0.4, 1.2, size=3)
            cx = rng.uniform(-2.0, 2.0)
            cz = rng.uniform(1.5, 3.5)
            blo = np.array([cx - size[0] / 2, hi[1] - size[1], cz - size[2] / 2])
            bhi = np.array([cx + size[0] / 2, hi[1], cz + size[2] / 2])
            boxes.append((blo, bhi))
        return Room(lo, hi, boxes, Texture.draw(rng))


def _pixel_rays():
    u, v = np.meshgrid(np.arange(CAM_W, dtype=np.float64),
                       np.arange(CAM_H, dtype=np.float64))
    d = np.stack([(u - CAM_CX) / CAM_F, (v - CAM_CY) / CAM_F, np.ones_like(u)], axis=-1)
    return d.reshape(-1, 3)          # camera-frame ray with unit z component


def render(room, G, rng, depth_noise=0.01, dmin=0.5, dmax=5.0):
    """Ray-cast one VGA frame from camera pose G (camera-to-world, 4x4).

    Returns per pixel (row-major, H*W): camera-frame noisy points [P,3],
    world surface points [P,3], validity mask [P], and the intensity image
    gradient magnitude plus the two gradient label channels.
    """
    dcam = _pixel_rays()
    R, o = G[:3, :3], G[:3, 3]
    dw = dcam @ R.T                                   # world-frame ray directions
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / dw
        # exit distance from the room interior
        t_hi = (room.hi[None, :] - o[None, :]) * inv
        t_lo = (room.lo[None, :] - o[None, :]) * inv
        t_exit = np.where(dw > 0, t_hi, np.where(dw < 0, t_lo, np.inf)).min(axis=1)
        s = t_exit
        for blo, bhi in room.boxes:
            t1 = (blo[None, :] - o[None, :]) * inv
            t2 = (bhi[None, :] - o[None, :]) * inv
            tn = np.minimum(t1, t2)
            tf = np.maximum(t1, t2)
            tn = np.where(np.isnan(tn), -np.inf, tn).max(axis=1)
            tf = np.where(np.isnan(tf), np.inf, tf).min(axis=1)
            hit = (tn <= tf) & (tn > 0)
            s = np.where(hit & (tn < s), tn, s)
    valid = np.isfinite(s) & (s >= dmin) & (s <= dmax)
    s = np.where(valid, s, 1.0)
    world = o[None, :] + s[:, None] * dw
    s_noisy = s * (1.0 + depth_noise * rng.standard_normal(s.shape))
    cam = s_noisy[:, None] * dcam
    col = room.tex.colour(world)
    inten = col.mean(axis=1).reshape(CAM_H, CAM_W)
    gv_img, gu_img = np.gradient(inten)               # per pixel, central differences
    gu = gu_img.reshape(-1)
    gv = gv_img.reshape(-1)
    feat = np.concatenate([col,
                           (0.5 + 0.5 * np.tanh(gu / 0.05))[:, None],
                           (0.5 + 0.5 * np.tanh(gv / 0.05))[:, None]], axis=1)
    gmag = np.hypot(gu, gv)
    return cam, world, valid, feat, gmag


def _select(valid, gmag, n, rng, mode):
    idx = np.flatnonzero(valid)
    if mode == "gradient":
        # top-n by |grad I|, ties broken by pixel index (stable sort)
        order = np.argsort(-gmag[idx], kind="stable")
        return np.sort(idx[order[:n]])
    if mode == "random":
        if n >= idx.size:
            return idx
        return np.sort(rng.choice(idx, size=n, replace=False))
    raise ValueError(mode)


def rgbd_pair(n_src=30000, n_tgt=None, seed=2, theta_max_deg=5.0, t_max=0.05,
              select="gradient", depth_noise=0.01):
    """Two synthetic RGB-D frames of one seeded room.

    The source camera is at the world origin, the target camera at a seeded
    pose G (theta <= theta_max, |t| <= t_max); each frame has its own depth
    noise (relative standard deviation depth_noise) and its own point
    selection.  T_true = G maps target-frame points onto source-frame points.
    """
    if n_tgt is None:
        n_tgt = n_src
    rng = np.random.default_rng(seed)
    room = Room.draw(rng)
    G = random_motion(rng, theta_max_deg, t_max)
    out = []
    for pose, n in ((np.eye(4), n_src), (G, n_tgt)):
        cam, _, valid, feat, gmag = render(room, pose, rng, depth_noise=depth_noise)
        sel = _select(valid, gmag, n, rng, select)
        out.append((cam[sel].astype(np.float32), feat[sel].astype(np.float32)))
    (sx, sf), (tx, tf) = out
    return CloudPair(sx, sf, tx, tf, G.copy(),
                     dict(kind="rgbd", seed=seed, n_src=len(sx), n_tgt=len(tx),
                          select=select, G=G))


def batched_sizes(count=256, seed0=4000, lo=5000, hi=60000):
    """Per-request (seed, n_src, n_tgt) for the batched workload."""
    out = []
    for k in range(count):
        rng = np.random.default_rng(seed0 + k + 1_000_000)
        out.append((seed0 + k, int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1))))
    return out


def serving_stream(rate, window_s=10.0, seed=5, median=20000, shape=1.0,
                   nmin=1000, nmax=300000):
    """Poisson arrival times and lognormal cloud sizes for the serving load.

    Returns a list of (arrival_s, request_seed, n_src, n_tgt).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    k = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= window_s:
            break
        ns, nt = (int(np.clip(round(math.exp(math.log(median) + shape * rng.standard_normal())),
                              nmin, nmax)) for _ in range(2))
        out.append((t, 5000 + k, ns, nt))
        k += 1
    return out


def default_schedule(n_stages=4, iters_per_stage=25, ell0=0.2, ell1=0.05):
    """Geometric length-scale annealing ell0 -> ell1 over n_stages stages."""
    if n_stages == 1:
        return [iters_per_stage], [ell0]
    ells = [ell0 * (ell1 / ell0) ** (s / (n_stages - 1)) for s in range(n_stages)]
    return [iters_per_stage] * n_stages, ells


# --------------------------------------------------------------------------
# RGB-D images (input of the device front end) and frame sequences
# --------------------------------------------------------------------------
@dataclass
class RGBDFrame:
    depth: np.ndarray          # [H, W] float32 metres, NaN where the ray has no valid return
    rgb: np.ndarray            # [H, W, 3] float32 colour in [0, 1]
    pose: np.ndarray           # camera-to-world 4x4 (ground truth)
    fx: float = CAM_F
    fy: float = CAM_F
    cx: float = CAM_CX
    cy: float = CAM_CY
    dmin: float = 0.5
    dmax: float = 5.0


def render_images(room, G, rng, depth_noise=0.01, dmin=0.5, dmax=5.0):
    """One VGA frame from camera pose G as images: depth along the optical
    axis with 1% multiplicative noise (NaN outside [dmin, dmax] or without a
    surface) and the colour of the world surface point."""
    cam, _, valid, feat, _ = render(room, G, rng, depth_noise=depth_noise, dmin=dmin, dmax=dmax)
    depth = np.where(valid, cam[:, 2], np.nan).astype(np.float32).reshape(CAM_H, CAM_W)
    rgb = feat[:, :3].astype(np.float32).reshape(CAM_H, CAM_W, 3)
    return RGBDFrame(depth, rgb, G.copy(), dmin=dmin, dmax=dmax)


def rgbd_frame_pair(seed=2, theta_max_deg=5.0, t_max=0.05):
    """The two frames of the RGB-D pair workload as images (same room and
    motion draw order as rgbd_pair with the same seed: source camera at the
    origin, target camera at G)."""
    rng = np.random.default_rng(seed)
    room = Room.draw(rng)
    G = random_motion(rng, theta_max_deg, t_max)
    return render_images(room, np.eye(4), rng), render_images(room, G, rng), G


def rgbd_sequence(n_frames=30, seed=9, step_deg=1.0, step_m=0.02, depth_noise=0.01):
    """A hand-held-like camera path through one seeded room: each frame moves
    by a smooth random rotation (about step_deg) and translation (about
    step_m) from the previous one.  Returns the frames (ground-truth poses in
    .pose, camera-to-world)."""
    rng = np.random.default_rng(seed)
    room = Room.draw(rng)
    frames = []
    G = np.eye(4)
    w = rng.normal(0.0, 1.0, 3)
    v = rng.normal(0.0, 1.0, 3)
    for k in range(n_frames):
        frames.append(render_images(room, G, rng, depth_noise=depth_noise))
        # slowly varying angular and linear velocity
        w = 0.8 * w + 0.2 * rng.normal(0.0, 1.0, 3)
        v = 0.8 * v + 0.2 * rng.normal(0.0, 1.0, 3)
        ang = math.radians(step_deg) * w / max(np.linalg.norm(w), 1e-12)
        R = rotation_axis_angle(ang / max(np.linalg.norm(ang), 1e-12), np.linalg.norm(ang))
        t = step_m * v / max(np.linalg.norm(v), 1e-12)
        M = np.eye(4)
        M[:3, :3] = R
        M[:3, 3] = t
        G = G @ M
    return frames
