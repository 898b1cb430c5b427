"""Frame-to-frame RGB-D odometry on the library (the paper's application,
Sec. VII-B): every frame goes through the device front end once; each new
frame is registered against the previous one, and the relative motions are
chained into a trajectory.

This module only orders calls and composes 4x4 poses on the host; the front
end and the registrations run in the HIP library.

Conventions: a frame's pose G_k is camera-to-world.  Registering frame k+1
(target) against frame k (source) returns T with T z = x for a point seen as
z in frame k+1 and as x in frame k, i.e. T = G_k^-1 G_{k+1}; the trajectory
is G_{k+1} = G_k T.

Errors per frame pair (the relative errors of Sec. VII-B): with the estimate
T and the truth T* = G_k^-1 G_{k+1}, the rotation error is the angle of
R R*^T and the translation error |t - t*|.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, List, Optional

import numpy as np


def relative_truth(G0, G1):
    """T* = G0^-1 G1 for camera-to-world poses."""
    R0, t0 = G0[:3, :3], G0[:3, 3]
    out = np.eye(4)
    out[:3, :3] = R0.T @ G1[:3, :3]
    out[:3, 3] = R0.T @ (G1[:3, 3] - t0)
    return out


def pose_errors(T, T_true):
    """(rotation angle in degrees, translation error in m) of T against T_true."""
    E = T[:3, :3] @ T_true[:3, :3].T
    ang = float(np.degrees(np.arccos(np.clip((np.trace(E) - 1.0) / 2.0, -1.0, 1.0))))
    return ang, float(np.linalg.norm(T[:3, 3] - T_true[:3, 3]))


@dataclass
class OdometryResult:
    relative: List[np.ndarray]          # estimated T for each frame pair
    trajectory: List[np.ndarray]        # chained camera-to-world poses (frame 0 at its true pose)
    rot_err_deg: np.ndarray             # per pair
    trans_err_m: np.ndarray
    iterations: List[int]
    wall_ms: List[float]                # per pair: front end of the new frame + registration

    def cdf(self, q=(50, 90, 99)):
        """Percentiles of the relative errors (the cumulative distributions of
        the paper's odometry figure)."""
        return {"rot_deg": {p: float(np.percentile(self.rot_err_deg, p)) for p in q},
                "trans_m": {p: float(np.percentile(self.trans_err_m, p)) for p in q}}


def run(frames, register: Callable, frontend: Callable, init: str = "identity") -> OdometryResult:
    """Chain frame-to-frame registrations over `frames` (objects with depth,
    rgb, intrinsics and a ground-truth .pose).

    frontend(frame) -> cloud; register(src_cloud, tgt_cloud, T0) -> (T, iters).
    init: "identity" (the paper's choice: every registration starts at the
    identity) or "constant_velocity" (start at the previous estimate).
    """
    import time
    if init not in ("identity", "constant_velocity"):
        raise ValueError(init)
    prev = frontend(frames[0])
    traj = [frames[0].pose.copy()]
    rel, rot, trans, iters, wall = [], [], [], [], []
    T0 = np.eye(4)
    for k in range(1, len(frames)):
        t0 = time.perf_counter()
        cur = frontend(frames[k])
        T, it = register(prev, cur, T0)
        wall.append((time.perf_counter() - t0) * 1e3)
        rel.append(T)
        traj.append(traj[-1] @ T)
        a, b = pose_errors(T, relative_truth(frames[k - 1].pose, frames[k].pose))
        rot.append(a)
        trans.append(b)
        iters.append(it)
        prev = cur
        if init == "constant_velocity":
            T0 = T
    return OdometryResult(rel, traj, np.array(rot), np.array(trans), iters, wall)


def run_on_device(ctx, frames, params, k: int = 30000, init: str = "identity",
                  device: Optional[object] = None) -> OdometryResult:
    """run() with the library: frames are uploaded once as torch tensors, the
    clouds stay on the device between the front end and the registrations."""
    import torch
    dev = torch.device("cuda:0") if device is None else device

    def frontend(f):
        d = torch.from_numpy(f.depth).to(dev)
        c = torch.from_numpy(f.rgb).to(dev)
        return ctx.frontend(d, c, k, f.fx, f.fy, f.cx, f.cy, f.dmin, f.dmax)

    def register(src, tgt, T0):
        out = ctx.register(src[0], src[1], tgt[0], tgt[1], params, T0=T0)
        return out["T"], out["iters"]

    return run(frames, register, frontend, init=init)


def run_served(ctx, frames, params, k: int = 30000, init: str = "identity",
               device: Optional[object] = None) -> OdometryResult:
    """run() through the serving path: every frame goes through the device
    front end once; the frame-pair registrations are submitted to the
    context's continuous-batching scheduler (cvo_submit) and collected with
    cvo_poll.  With init "identity" each pair is submitted as soon as its
    target frame's front end is done, so the scheduler registers it while
    the next frames are processed, and the pairs share batches; with
    "constant_velocity" each pair waits for the previous estimate (its
    initial pose).  The clouds stay on the device and are kept alive until
    their tickets are polled."""
    import time
    import torch
    if init not in ("identity", "constant_velocity"):
        raise ValueError(init)
    dev = torch.device("cuda:0") if device is None else device
    t0 = time.perf_counter()

    def frontend(f):
        d = torch.from_numpy(f.depth).to(dev)
        c = torch.from_numpy(f.rgb).to(dev)
        return ctx.frontend(d, c, k, f.fx, f.fy, f.cx, f.cy, f.dmin, f.dmax)

    def collect(tk):
        out = ctx.poll(tk)
        if out["rc"] < 0:
            raise RuntimeError(f"registration failed: {out['rc']}")
        rel.append(out["T"])
        iters.append(out["iters"])
        return out["T"]

    rel, iters = [], []
    clouds = [frontend(frames[0])] if frames else []
    if init == "identity":
        tickets = []
        for q in range(1, len(frames)):
            clouds.append(frontend(frames[q]))
            tickets.append(ctx.submit(clouds[q - 1][0], clouds[q - 1][1], clouds[q][0], clouds[q][1], params))
        for tk, keep in tickets:
            collect(tk)
    else:
        T0 = np.eye(4)
        for q in range(1, len(frames)):
            clouds.append(frontend(frames[q]))
            tk, keep = ctx.submit(clouds[q - 1][0], clouds[q - 1][1], clouds[q][0], clouds[q][1], params, T0=T0)
            T0 = collect(tk)
    wall = (time.perf_counter() - t0) * 1e3
    traj = [frames[0].pose.copy()]
    rot, trans = [], []
    for q, T in enumerate(rel):
        traj.append(traj[-1] @ T)
        a, b = pose_errors(T, relative_truth(frames[q].pose, frames[q + 1].pose))
        rot.append(a)
        trans.append(b)
    per = wall / max(1, len(rel))
    return OdometryResult(rel, traj, np.array(rot), np.array(trans), iters, [per] * len(rel))
