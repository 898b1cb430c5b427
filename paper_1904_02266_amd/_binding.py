"""ctypes binding of the C ABI in include/cvo.h (argument marshalling only).

Every step of the registration runs in the HIP library; this module only
turns NumPy arrays / torch tensors into cvo_cloud structs and back.  If the
built library is missing, loading fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libcvo.so")

CVO_OK = 0
CVO_PENDING = 1
CVO_EINVAL = -1
CVO_ENOMEM = -2
CVO_EBUSY = -3
CVO_ENOOVERLAP = -4
CVO_EDEVICE = -5
CVO_ENOTFOUND = -6
CVO_FP32_KAHAN = 0
CVO_FP64 = 1
CVO_STEP_FIXED = 0
CVO_STEP_QUARTIC = 1
CVO_STEP_CONJUGATE = 2
STEP_RULES = {"fixed": CVO_STEP_FIXED, "quartic": CVO_STEP_QUARTIC, "conjugate": CVO_STEP_CONJUGATE}
# subgroups of SE(3) for Params.dof_mask (bits: rotation x, y, z, translation x, y, z)
DOF_SE3, DOF_SE2, DOF_SO3, DOF_R3 = 0x3F, 0x1C, 0x07, 0x38
TRACE_COLS = 26


class cvo_cloud(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("feat_dim", ctypes.c_int32),
                ("xyz", ctypes.c_void_p), ("feat", ctypes.c_void_p),
                ("on_device", ctypes.c_int32)]


class cvo_params(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("feat_scale", ctypes.c_double),
                ("a2", ctypes.c_double), ("b2", ctypes.c_double), ("eta", ctypes.c_double),
                ("cutoff_mult", ctypes.c_double), ("n_stages", ctypes.c_int32),
                ("stage_iters", ctypes.POINTER(ctypes.c_int32)),
                ("stage_ell", ctypes.POINTER(ctypes.c_double)),
                ("max_iters", ctypes.c_int32), ("tol", ctypes.c_double),
                ("precision", ctypes.c_int32), ("trace", ctypes.c_int32), ("step_rule", ctypes.c_int32),
                ("grad_tol", ctypes.c_double), ("kernel_floor", ctypes.c_double), ("dof_mask", ctypes.c_int32),
                ("stage_tol", ctypes.c_double), ("work_item_min", ctypes.c_int32),
                ("work_items_max", ctypes.c_int32)]


class cvo_serving_counters(ctypes.Structure):
    _fields_ = [("pending", ctypes.c_int64), ("active", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("hbm_in_use", ctypes.c_uint64), ("hbm_budget", ctypes.c_uint64),
                ("hbm_peak", ctypes.c_uint64), ("graph_chunks", ctypes.c_int64)]


class cvo_rgbd_frame(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("depth", ctypes.c_void_p), ("rgb", ctypes.c_void_p),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("dmin", ctypes.c_double), ("dmax", ctypes.c_double), ("on_device", ctypes.c_int32)]


class cvo_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("F", ctypes.c_double), ("omega", ctypes.c_double * 3), ("v", ctypes.c_double * 3),
                ("gpu_ms", ctypes.c_double), ("wall_ms", ctypes.c_double),
                ("pairs_within", ctypes.c_uint64), ("pairs_examined", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64)]

    def as_dict(self):
        return dict(status=self.status, iters=self.iters, converged=bool(self.converged), F=self.F,
                    omega=np.array(self.omega[:]), v=np.array(self.v[:]), gpu_ms=self.gpu_ms,
                    wall_ms=self.wall_ms, pairs_within=int(self.pairs_within),
                    pairs_examined=int(self.pairs_examined), device_bytes=int(self.device_bytes))


_lib = None


def load():
    """Load the built HIP library; raise if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(build it with: python -m paper_1904_02266_amd.build)")
    # One HIP runtime per process: torch ships its own libamdhip64.so.7.  Loading
    # torch first makes the library bind to that already-loaded runtime (same
    # soname), so device pointers and streams are shared with torch.
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover - the library also works without torch
        pass
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i32, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    L.cvo_create.argtypes = [ctypes.c_int, u64, ctypes.c_int, P(vp)]
    L.cvo_destroy.argtypes = [vp]
    L.cvo_set_stream.argtypes = [vp, vp]
    L.cvo_eval.argtypes = [vp, P(cvo_cloud), P(cvo_cloud), P(cvo_params), P(dbl), P(dbl), P(dbl), P(dbl)]
    L.cvo_eval_static.argtypes = [vp, P(cvo_cloud), P(cvo_cloud), P(cvo_params), P(dbl), P(dbl), P(dbl), P(dbl)]
    L.cvo_eval_targets.argtypes = [vp, P(cvo_cloud), P(cvo_cloud), P(cvo_params), P(dbl), i32,
                                   P(i32), P(dbl)]
    L.cvo_register.argtypes = [vp, P(cvo_cloud), P(cvo_cloud), P(cvo_params), P(dbl), P(dbl),
                               P(cvo_result)]
    L.cvo_submit.argtypes = [vp, P(cvo_cloud), P(cvo_cloud), P(cvo_params), P(dbl), P(u64)]
    L.cvo_poll.argtypes = [vp, u64, i32, P(dbl), P(cvo_result)]
    L.cvo_trace.argtypes = [vp, u64, P(dbl), i32]
    L.cvo_set_profiling.argtypes = [vp, i32]
    L.cvo_kernel_stats.argtypes = [vp, i32, P(ctypes.c_int64), P(dbl), P(dbl), P(dbl), P(u64)]
    L.cvo_quartic.argtypes = [vp, P(cvo_cloud), P(cvo_cloud), P(cvo_params), P(dbl), P(dbl), P(dbl), P(dbl)]
    L.cvo_quartic_step.argtypes = [P(dbl), P(dbl)]
    L.cvo_quartic_step_bounded.argtypes = [P(dbl), dbl, P(dbl)]
    L.cvo_frontend.argtypes = [vp, P(cvo_rgbd_frame), i32, vp, vp, P(i32)]
    L.cvo_serving_stats.argtypes = [vp, P(cvo_serving_counters)]
    L.cvo_set_queue_limit.argtypes = [vp, ctypes.c_int64]
    L.cvo_tuning.argtypes = [vp, i32, i32, i32, P(i32), P(i32), P(i32)]
    L.cvo_set_graphs.argtypes = [vp, i32]
    L.cvo_strerror.argtypes = [ctypes.c_int]
    L.cvo_strerror.restype = ctypes.c_char_p
    L.cvo_last_error.argtypes = [vp]
    L.cvo_last_error.restype = ctypes.c_char_p
    for name in ("cvo_create", "cvo_destroy", "cvo_set_stream", "cvo_eval", "cvo_eval_targets",
                 "cvo_register", "cvo_submit", "cvo_poll", "cvo_trace", "cvo_set_profiling",
                 "cvo_kernel_stats", "cvo_quartic", "cvo_quartic_step", "cvo_frontend", "cvo_serving_stats",
                 "cvo_set_queue_limit", "cvo_eval_static", "cvo_tuning", "cvo_set_graphs",
                 "cvo_quartic_step_bounded"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


EXPORTED = ("cvo_create", "cvo_destroy", "cvo_set_stream", "cvo_eval", "cvo_eval_targets",
            "cvo_register", "cvo_submit", "cvo_poll", "cvo_trace", "cvo_set_profiling",
            "cvo_kernel_stats", "cvo_quartic", "cvo_quartic_step", "cvo_frontend", "cvo_serving_stats",
            "cvo_set_queue_limit", "cvo_eval_static", "cvo_tuning", "cvo_set_graphs",
            "cvo_quartic_step_bounded", "cvo_strerror", "cvo_last_error")


class CvoError(RuntimeError):
    def __init__(self, code, msg=""):
        L = load()
        text = L.cvo_strerror(code).decode()
        super().__init__(f"cvo error {code} ({text}) {msg}".strip())
        self.code = code


@dataclass
class Params:
    sigma: float = 0.1
    feat_scale: float = 0.2
    a2: float = -1.0
    b2: float = 1.0
    eta: float = 1.0
    cutoff_mult: float = 0.0
    stage_iters: Sequence[int] = field(default_factory=tuple)
    stage_ell: Sequence[float] = field(default_factory=lambda: (0.1,))
    max_iters: int = 50
    tol: float = 0.0
    precision: str = "fp32"
    trace: bool = False
    step_rule: str = "fixed"
    grad_tol: float = 0.0
    kernel_floor: float = 0.0
    dof_mask: int = 0
    stage_tol: float = 0.0       # > 0: a stage ends early once |tau d| < stage_tol
    work_item_min: int = 0       # 0: the context's tuning table
    work_items_max: int = 0

    def to_c(self):
        ns = len(self.stage_ell)
        si = (ctypes.c_int32 * max(1, ns))(*([int(v) for v in self.stage_iters] + [0] * (ns - len(self.stage_iters))))
        se = (ctypes.c_double * max(1, ns))(*[float(v) for v in self.stage_ell])
        p = cvo_params(self.sigma, self.feat_scale, self.a2, self.b2, self.eta, self.cutoff_mult, ns,
                       ctypes.cast(si, ctypes.POINTER(ctypes.c_int32)),
                       ctypes.cast(se, ctypes.POINTER(ctypes.c_double)), self.max_iters, self.tol,
                       CVO_FP64 if self.precision == "fp64" else CVO_FP32_KAHAN, 1 if self.trace else 0,
                       STEP_RULES[self.step_rule], self.grad_tol, self.kernel_floor, self.dof_mask,
                       self.stage_tol, self.work_item_min, self.work_items_max)
        return p, (si, se)


def params_planes(**kw):
    """Three-plane brute-force workload: ell = 0.1 fixed, all pairs, 50 steps."""
    base = dict(stage_ell=(0.1,), max_iters=50, cutoff_mult=0.0)
    base.update(kw)
    return Params(**base)


def params_table1(**kw):
    """The TUM-experiment parameters of Table 1: ell 0.15, 0.10 after iteration
    3, 0.06 after 10, 0.03 after 20; sigma 0.1; kernel values below 1e-3
    dropped; transformation and gradient-norm thresholds 1e-5 and 5e-5; the
    quartic step.  (The colour inner-product scale and the minimum step length
    are not taken over: see the readings of the step rule and of the labels.)"""
    base = dict(stage_ell=(0.15, 0.10, 0.06, 0.03), stage_iters=(4, 7, 10), max_iters=200, sigma=0.1,
                kernel_floor=1e-3, tol=1e-5, grad_tol=5e-5, step_rule="quartic")
    base.update(kw)
    return Params(**base)


def params_rgbd(**kw):
    """RGB-D frame workload: cutoff 3 ell, ell annealed 0.2 -> 0.05 m geometrically
    over 4 stages of 25 iterations (100 iterations)."""
    ells = tuple(0.2 * (0.25 ** (s / 3.0)) for s in range(4))
    base = dict(stage_ell=ells, stage_iters=(25, 25, 25), max_iters=100, cutoff_mult=3.0)
    base.update(kw)
    return Params(**base)


class _Cloud:
    """Keeps the buffers of one cloud alive while the call runs."""

    def __init__(self, xyz, feat):
        self.keep = []
        try:
            import torch
            is_t = isinstance(xyz, torch.Tensor)
        except ImportError:  # pragma: no cover
            is_t = False
        if is_t:
            import torch
            if xyz.is_cuda != feat.is_cuda:
                raise ValueError("xyz and feat must live on the same device")
            xyz = xyz.to(torch.float32).contiguous()
            feat = feat.to(torch.float32).contiguous()
            if xyz.dim() != 2 or xyz.shape[1] != 3 or feat.dim() != 2 or feat.shape[0] != xyz.shape[0]:
                raise ValueError("xyz must be [n,3] and feat [n,F]")
            self.keep = [xyz, feat]
            self.on_device = 1 if xyz.is_cuda else 0
            self.c = cvo_cloud(xyz.shape[0], feat.shape[1], xyz.data_ptr(), feat.data_ptr(), self.on_device)
        else:
            xyz = np.ascontiguousarray(xyz, dtype=np.float32)
            feat = np.ascontiguousarray(feat, dtype=np.float32)
            if xyz.ndim != 2 or xyz.shape[1] != 3 or feat.ndim != 2 or feat.shape[0] != xyz.shape[0]:
                raise ValueError("xyz must be [n,3] and feat [n,F]")
            self.keep = [xyz, feat]
            self.on_device = 0
            self.c = cvo_cloud(xyz.shape[0], feat.shape[1], xyz.ctypes.data, feat.ctypes.data, 0)


def _pose(T):
    T = np.ascontiguousarray(np.asarray(T, dtype=np.float64).reshape(16))
    return T, T.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def quartic_step(coef, tmax=None):
    """The quartic rule's step for coefficients (F, A1..A4): the maximiser over
    t > 0 (t <= tmax when given) of A1 t + ... + A4 t^4 among its local maxima,
    or None when it has none there (host code of the library, the rule the
    step kernel applies)."""
    L = load()
    c = (ctypes.c_double * 5)(*[float(a) for a in coef])
    t = ctypes.c_double()
    if tmax is None:
        rc = L.cvo_quartic_step(c, ctypes.byref(t))
    else:
        rc = L.cvo_quartic_step_bounded(c, float(tmax), ctypes.byref(t))
    if rc < 0:
        raise CvoError(rc, "cvo_quartic_step")
    return t.value if rc == 1 else None


class Context:
    """One library context on one HIP device."""

    def __init__(self, device=0, hbm_budget=0, max_slots=256):
        self.L = load()
        h = ctypes.c_void_p()
        rc = self.L.cvo_create(device, hbm_budget, max_slots, ctypes.byref(h))
        if rc != 0:
            raise CvoError(rc, "cvo_create")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            self.L.cvo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc < 0:
            raise CvoError(rc, f"{what}: {self.L.cvo_last_error(self.h).decode()}")
        return rc

    def _sync_stream(self, clouds):
        """Device inputs: run on torch's current stream, ordered after the work
        queued there.  torch's legacy default stream cannot carry that order
        (the library then uses its own non-blocking stream), so it is
        synchronized first."""
        if any(c.on_device for c in clouds):
            import torch
            cur = torch.cuda.current_stream(self.device)
            if cur.cuda_stream == 0:
                cur.synchronize()
            self.L.cvo_set_stream(self.h, ctypes.c_void_p(cur.cuda_stream))
        else:
            self.L.cvo_set_stream(self.h, None)

    def set_graphs(self, on=True):
        """Replay the iteration chunks of cvo_register and of the batched
        scheduler as HIP graphs (see cvo_set_graphs)."""
        self._check(self.L.cvo_set_graphs(self.h, 1 if on else 0), "set_graphs")

    def set_profiling(self, on=True):
        self._check(self.L.cvo_set_profiling(self.h, 1 if on else 0), "set_profiling")

    def kernel_stats(self, reset=False):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        prep = ctypes.c_double()
        quart = ctypes.c_double()
        pairs = ctypes.c_uint64()
        self._check(self.L.cvo_kernel_stats(self.h, 1 if reset else 0, ctypes.byref(n), ctypes.byref(ms),
                                            ctypes.byref(prep), ctypes.byref(quart), ctypes.byref(pairs)),
                    "kernel_stats")
        return dict(launches=n.value, ms=ms.value, prepare_ms=prep.value, quartic_ms=quart.value,
                    pairs=pairs.value)

    def eval(self, src_xyz, src_feat, tgt_xyz, tgt_feat, T, params: Params):
        s, t = _Cloud(src_xyz, src_feat), _Cloud(tgt_xyz, tgt_feat)
        self._sync_stream([s, t])
        p, keep = params.to_c()
        Ta, Tp = _pose(T)
        F = ctypes.c_double()
        w = (ctypes.c_double * 3)()
        v = (ctypes.c_double * 3)()
        self._check(self.L.cvo_eval(self.h, ctypes.byref(s.c), ctypes.byref(t.c), ctypes.byref(p), Tp,
                                    ctypes.byref(F), w, v), "cvo_eval")
        return np.array([F.value, *w[:], *v[:]])

    def eval_static(self, src_xyz, src_feat, tgt_xyz, tgt_feat, T, params: Params):
        """eval() through cvo_eval_static: no allocation inside the library call
        (the device buffers come from the library's per-device static array)."""
        s, t = _Cloud(src_xyz, src_feat), _Cloud(tgt_xyz, tgt_feat)
        self._sync_stream([s, t])
        p, keep = params.to_c()
        Ta, Tp = _pose(T)
        F = ctypes.c_double()
        w = (ctypes.c_double * 3)()
        v = (ctypes.c_double * 3)()
        self._check(self.L.cvo_eval_static(self.h, ctypes.byref(s.c), ctypes.byref(t.c), ctypes.byref(p), Tp,
                                           ctypes.byref(F), w, v), "cvo_eval_static")
        return np.array([F.value, *w[:], *v[:]])

    def frontend(self, depth, rgb, k, fx, fy, cx, cy, dmin=0.5, dmax=5.0):
        """Semi-dense cloud of one RGB-D frame: (xyz [n,3], feat [n,5]) as float32,
        NumPy arrays for host images, torch tensors on the device for device ones."""
        try:
            import torch
            is_t = isinstance(depth, torch.Tensor) and depth.is_cuda
        except ImportError:  # pragma: no cover
            is_t = False
        if is_t:
            import torch
            depth = depth.to(torch.float32).contiguous()
            rgb = rgb.to(torch.float32).contiguous()
            H, W = depth.shape
            if tuple(rgb.shape) != (H, W, 3) or not rgb.is_cuda:
                raise ValueError("rgb must be [H,W,3] on the same device as depth")
            xyz = torch.empty((k, 3), dtype=torch.float32, device=depth.device)
            feat = torch.empty((k, 5), dtype=torch.float32, device=depth.device)
            self.L.cvo_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))
            fr = cvo_rgbd_frame(W, H, depth.data_ptr(), rgb.data_ptr(), fx, fy, cx, cy, dmin, dmax, 1)
            xp, fp = xyz.data_ptr(), feat.data_ptr()
        else:
            depth = np.ascontiguousarray(depth, dtype=np.float32)
            rgb = np.ascontiguousarray(rgb, dtype=np.float32)
            H, W = depth.shape
            if rgb.shape != (H, W, 3):
                raise ValueError("rgb must be [H,W,3]")
            xyz = np.zeros((k, 3), np.float32)
            feat = np.zeros((k, 5), np.float32)
            self.L.cvo_set_stream(self.h, None)
            fr = cvo_rgbd_frame(W, H, depth.ctypes.data, rgb.ctypes.data, fx, fy, cx, cy, dmin, dmax, 0)
            xp, fp = xyz.ctypes.data, feat.ctypes.data
        n = ctypes.c_int32()
        self._check(self.L.cvo_frontend(self.h, ctypes.byref(fr), k, ctypes.c_void_p(xp), ctypes.c_void_p(fp),
                                        ctypes.byref(n)), "cvo_frontend")
        return xyz[: n.value], feat[: n.value]

    def quartic(self, src_xyz, src_feat, tgt_xyz, tgt_feat, T, omega, v, params: Params):
        """F, A1..A4 of the fourth-order model of G(t) = F(h exp(t (omega, v))) at T."""
        s, t = _Cloud(src_xyz, src_feat), _Cloud(tgt_xyz, tgt_feat)
        self._sync_stream([s, t])
        p, keep = params.to_c()
        Ta, Tp = _pose(T)
        w = (ctypes.c_double * 3)(*[float(a) for a in omega])
        u = (ctypes.c_double * 3)(*[float(a) for a in v])
        coef = (ctypes.c_double * 5)()
        self._check(self.L.cvo_quartic(self.h, ctypes.byref(s.c), ctypes.byref(t.c), ctypes.byref(p), Tp, w, u,
                                       coef), "cvo_quartic")
        return np.array(coef[:])

    def eval_targets(self, src_xyz, src_feat, tgt_xyz, tgt_feat, T, params: Params, sel=None):
        s, t = _Cloud(src_xyz, src_feat), _Cloud(tgt_xyz, tgt_feat)
        self._sync_stream([s, t])
        p, keep = params.to_c()
        Ta, Tp = _pose(T)
        if sel is None:
            out = np.zeros((t.c.n, 7))
            rc = self.L.cvo_eval_targets(self.h, ctypes.byref(s.c), ctypes.byref(t.c), ctypes.byref(p), Tp, 0,
                                         None, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        else:
            sel = np.ascontiguousarray(sel, dtype=np.int32)
            out = np.zeros((sel.size, 7))
            rc = self.L.cvo_eval_targets(self.h, ctypes.byref(s.c), ctypes.byref(t.c), ctypes.byref(p), Tp,
                                         sel.size, sel.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        self._check(rc, "cvo_eval_targets")
        return out

    def register(self, src_xyz, src_feat, tgt_xyz, tgt_feat, params: Params, T0=None, check=True):
        s, t = _Cloud(src_xyz, src_feat), _Cloud(tgt_xyz, tgt_feat)
        self._sync_stream([s, t])
        p, keep = params.to_c()
        Ta, Tp = _pose(np.eye(4) if T0 is None else T0)
        Tout = np.zeros(16)
        res = cvo_result()
        rc = self.L.cvo_register(self.h, ctypes.byref(s.c), ctypes.byref(t.c), ctypes.byref(p), Tp,
                                 Tout.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(res))
        if check:
            self._check(rc, "cvo_register")
        out = res.as_dict()
        out["rc"] = rc
        out["T"] = Tout.reshape(4, 4)
        return out

    def register_planar(self, src_xy, src_feat, tgt_xy, tgt_feat, params: Params, T0=None, check=True):
        """Registration of planar clouds on SE(2) (the n = 2 case of the
        general-n gradient): points [n, 2] are passed as (x, y, 0) and the flow
        runs on the subgroup of rotations about z and translations in the
        plane (dof_mask 0x1C), whose gradient is eq. flow's for n = 2.  T0 and
        the returned T are 3x3 (acting on target points)."""
        import dataclasses

        def lift(xy):
            xy = np.asarray(xy, dtype=np.float32)
            if xy.ndim != 2 or xy.shape[1] != 2:
                raise ValueError("planar points must be [n, 2]")
            return np.concatenate([xy, np.zeros((xy.shape[0], 1), np.float32)], axis=1)

        T4 = np.eye(4)
        if T0 is not None:
            T0 = np.asarray(T0, dtype=np.float64)
            T4[:2, :2] = T0[:2, :2]
            T4[:2, 3] = T0[:2, 2]
        out = self.register(lift(src_xy), src_feat, lift(tgt_xy), tgt_feat,
                            dataclasses.replace(params, dof_mask=DOF_SE2), T0=T4, check=check)
        T = np.eye(3)
        T[:2, :2] = out["T"][:2, :2]
        T[:2, 2] = out["T"][:2, 3]
        out["T"] = T
        return out

    def trace(self, cap=100000, ticket=0):
        """The per-iteration trace of the last register call (ticket 0) or of a
        finished batched ticket; None while that ticket is still running."""
        buf = np.zeros((cap, TRACE_COLS))
        rows = self._check(self.L.cvo_trace(self.h, ticket, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            cap), "cvo_trace")
        if rows == CVO_PENDING and ticket != 0:
            return None
        return buf[:rows]

    def tuning(self, n, m, cutoff=True):
        """(work_item_min, work_items_max, classes in the loaded table) for a request
        of n sources and m targets."""
        a, b_, t = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.L.cvo_tuning(self.h, n, m, 1 if cutoff else 0, ctypes.byref(a), ctypes.byref(b_),
                                      ctypes.byref(t)), "cvo_tuning")
        return a.value, b_.value, t.value

    def set_queue_limit(self, max_pending):
        self._check(self.L.cvo_set_queue_limit(self.h, int(max_pending)), "cvo_set_queue_limit")

    def submit(self, src_xyz, src_feat, tgt_xyz, tgt_feat, params: Params, T0=None):
        """Returns (ticket, keepalive); keep `keepalive` until the ticket is polled
        when passing device tensors (they are borrowed).  Device tensors are read
        later on the scheduler's stream: torch's current stream is synchronized
        first, so conversions queued on it (dtype, contiguity) are complete."""
        s, t = _Cloud(src_xyz, src_feat), _Cloud(tgt_xyz, tgt_feat)
        if s.on_device or t.on_device:
            import torch
            torch.cuda.current_stream(self.device).synchronize()
        p, keep = params.to_c()
        Ta, Tp = _pose(np.eye(4) if T0 is None else T0)
        tk = ctypes.c_uint64()
        self._check(self.L.cvo_submit(self.h, ctypes.byref(s.c), ctypes.byref(t.c), ctypes.byref(p), Tp,
                                      ctypes.byref(tk)), "cvo_submit")
        return tk.value, (s, t)

    def serving_stats(self):
        """Counters of the batched path: pending, active, completed, failed,
        hbm_in_use, hbm_budget, hbm_peak, graph_chunks."""
        st = cvo_serving_counters()
        self._check(self.L.cvo_serving_stats(self.h, ctypes.byref(st)), "cvo_serving_stats")
        return {f: getattr(st, f) for f, _ in cvo_serving_counters._fields_}

    def poll(self, ticket, wait_us=-1):
        Tout = np.zeros(16)
        res = cvo_result()
        rc = self.L.cvo_poll(self.h, ticket, wait_us, Tout.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             ctypes.byref(res))
        if rc == CVO_PENDING:
            return None
        out = res.as_dict()
        out["rc"] = rc
        out["T"] = Tout.reshape(4, 4)
        return out
